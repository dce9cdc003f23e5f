// Host gate-pass compilers. Both turn a program-order gate sequence into
// passes of groups on pairwise disjoint qubit sets; gates of different groups
// commute, so applying a pass group by group equals applying its gates in
// program order, and every column of a group is read and written once per
// pass whatever the number of gates on it.
//
// * WideBuilder (the tableau kernels): groups of up to WG_MAXQ qubits and
//   WG_MAXOPS micro-ops, placed as early as possible (a gate goes to the
//   latest pass holding one of its qubits, joining or merging their groups
//   there if the group stays within the limits, else to the next pass). A
//   random generator layer then needs well under one pass, because a group
//   keeps absorbing the following layers' gates on its qubits until its light
//   cone outgrows WG_MAXQ.
// * PassBuilder (the batched persistent kernel): groups of one or two qubits
//   and up to 16 4-bit micro-ops; any other overlap closes the pass.
#pragma once
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <deque>
#include <thread>
#include <vector>

#include "../../include/sq.h"
#include "sq_internal.h"

namespace sq {

inline bool is_two_qubit(u32 t) {
  return t == SQ_CX || t == SQ_CZ || t == SQ_CY || t == SQ_SWAP || t == SQ_ISWAP;
}

struct PassRange {
  u64 offset;  // first group (index into the group list or the offset table)
  u32 count;
  u64 bytes;   // algorithmic bytes of the pass: column reads + changed-column writes
};

// ============================================================== wide groups
inline u32 wide_type(u32 sq_type) {
  switch (sq_type) {
    case SQ_H: return WOP_H;
    case SQ_S: return WOP_S;
    case SQ_SDG: return WOP_SDG;
    case SQ_X: return WOP_X;
    case SQ_Y: return WOP_Y;
    case SQ_Z: return WOP_Z;
    case SQ_CX: return WOP_CX;
    case SQ_SWAP: return WOP_SWAP;
    default: return WOP_CZ;
  }
}

class WideBuilder {
 public:
  std::vector<u32> words;         // records of every emitted pass, in order
  std::vector<u32> offs;          // per group: word offset of its record
  std::vector<PassRange> passes;  // offset/count into offs

  // window: passes kept open at once (older ones are emitted and closed)
  void init(u32 n, u32 L, u32 window = 8) {
    n_ = n;
    L_ = L;
    window_ = std::max<u32>(window, 1);
    qs_.assign(n, QState{});
    lo_ = 0;
    open_.clear();
    words.clear();
    offs.clear();
    passes.clear();
  }

  void add(u32 type, u32 a, u32 b) {
    if (type == SQ_I) return;
    // products of the native rules, in time order: CY(a,b) = S_b CX(a,b)
    // S_b^dagger, iSWAP(a,b) = SWAP CZ (S_a S_b)
    if (type == SQ_CY) {
      add(SQ_SDG, b, 0);
      add(SQ_CX, a, b);
      add(SQ_S, b, 0);
      return;
    }
    if (type == SQ_ISWAP) {
      add(SQ_S, a, 0);
      add(SQ_S, b, 0);
      add(SQ_CZ, a, b);
      add(SQ_SWAP, a, b);
      return;
    }
    const bool two = is_two_qubit(type);
    QState &A = qs_[a];
    QState &Bq = qs_[two ? b : a];
    int64_t p = std::max<int64_t>(A.front, lo_);
    if (two) p = std::max<int64_t>(p, Bq.front);
    for (;; ++p) {
      while ((int64_t)(lo_ + open_.size()) <= p) {
        if (!pool_.empty()) {
          open_.push_back(std::move(pool_.back()));
          pool_.pop_back();
        } else {
          open_.emplace_back();
        }
      }
      std::vector<WG> &pass = open_[p - lo_];
      const int ga = A.front == p ? (int)A.grp : -1;
      const int gb = two && Bq.front == p ? (int)Bq.grp : -1;
      u32 size, ops;
      if (!two) {
        size = ga >= 0 ? pass[ga].nq : 1;
        ops = (ga >= 0 ? pass[ga].nops : 0) + 1;
      } else if (ga >= 0 && ga == gb) {
        size = pass[ga].nq;
        ops = pass[ga].nops + 1;
      } else {
        size = (ga >= 0 ? pass[ga].nq : 1) + (gb >= 0 ? pass[gb].nq : 1);
        ops = (ga >= 0 ? pass[ga].nops : 0) + (gb >= 0 ? pass[gb].nops : 0) + 1;
      }
      if (size > WG_MAXQ || ops > WG_MAXOPS) continue;
      int g = ga >= 0 ? ga : gb;
      if (g < 0) {
        pass.emplace_back();
        g = (int)pass.size() - 1;
      }
      if (two && ga >= 0 && gb >= 0 && ga != gb) merge(pass, ga, gb, p);
      const u32 sa = slot_of(pass[g], a, g, p);
      const u32 sb = two ? slot_of(pass[g], b, g, p) : 0;
      WG &G = pass[g];
      G.ops[G.nops++] = (uint16_t)(wide_type(type) | (sa << 4) | (sb << 8));
      break;
    }
    while (p - lo_ >= window_) emit_oldest();
  }

  // Close every open pass (measurement boundaries, end of input).
  void flush() {
    while (!open_.empty()) emit_oldest();
  }

 private:
  struct WG {
    uint8_t nq = 0, nops = 0;
    bool alive = true;
    u32 q[WG_MAXQ];
    uint16_t ops[WG_MAXOPS];
  };
  u32 n_ = 0, L_ = 0, window_ = 8;
  int64_t lo_ = 0;                     // index of the oldest open pass
  std::deque<std::vector<WG>> open_;   // open_[i] holds pass lo_ + i
  std::vector<std::vector<WG>> pool_;  // emptied pass vectors, storage kept
  // per qubit: the last pass holding it (-1 none), its group and slot there.
  // A gate on q is placed at a pass p >= front, so q is in the chosen group
  // exactly when front == p and grp is that group.
  struct QState {
    int64_t front = -1;
    u32 grp = 0, slot = 0;
  };
  std::vector<QState> qs_;

  u32 slot_of(WG &G, u32 q, int g, int64_t p) {
    QState &Q = qs_[q];
    if (Q.front == p && Q.grp == (u32)g) return Q.slot;
    G.q[G.nq] = q;
    Q.front = p;
    Q.grp = (u32)g;
    Q.slot = G.nq;
    return G.nq++;
  }

  // Append group gb (slots renumbered after ga's) to ga; their ops commute.
  // Members that already have gates in later passes keep pointing there.
  void merge(std::vector<WG> &pass, int ga, int gb, int64_t p) {
    WG &A = pass[ga];
    WG &B = pass[gb];
    const u32 base = A.nq;
    for (u32 i = 0; i < B.nq; ++i) {
      A.q[base + i] = B.q[i];
      QState &Q = qs_[B.q[i]];
      if (Q.front == p) {
        Q.grp = (u32)ga;
        Q.slot = base + i;
      }
    }
    A.nq = (uint8_t)(base + B.nq);
    for (u32 k = 0; k < B.nops; ++k) {
      const u32 op = B.ops[k];
      const u32 sa = ((op >> 4) & 15u) + base, sb = ((op >> 8) & 15u) + base;
      const bool two = (op & 15u) >= WOP_CX;
      A.ops[A.nops++] = (uint16_t)((op & 15u) | (sa << 4) | ((two ? sb : 0u) << 8));
    }
    B.alive = false;
    B.nq = B.nops = 0;
  }

  static u32 dirty(const WG &G) {
    u32 dx = 0, dz = 0;
    for (u32 k = 0; k < G.nops; ++k) {
      const u32 op = G.ops[k], t = op & 15u, a = (op >> 4) & 15u, b = (op >> 8) & 15u;
      switch (t) {
        case WOP_H: dx |= 1u << a; dz |= 1u << a; break;
        case WOP_S: case WOP_SDG: dz |= 1u << a; break;
        case WOP_CX: dx |= 1u << b; dz |= 1u << a; break;
        case WOP_CZ: dz |= (1u << a) | (1u << b); break;
        case WOP_SWAP: dx |= (1u << a) | (1u << b); dz |= (1u << a) | (1u << b); break;
        default: break;  // X, Y, Z change signs only
      }
    }
    return (dx << WH_DX_SHIFT) | (dz << WH_DZ_SHIFT);
  }

  void emit_oldest() {
    std::vector<WG> &pass = open_.front();
    const u64 first = offs.size();
    u64 bytes = 0;
    for (const WG &G : pass) {
      if (!G.alive || G.nops == 0) continue;
      const u32 d = dirty(G);
      offs.push_back((u32)words.size());
      words.push_back((u32)G.nq | ((u32)G.nops << WH_NOPS_SHIFT) | d);
      for (u32 i = 0; i < G.nq; ++i) words.push_back(G.q[i]);
      for (u32 k = 0; k < G.nops; k += 2)
        words.push_back((u32)G.ops[k] | (k + 1 < G.nops ? (u32)G.ops[k + 1] << 16 : 0u));
      bytes += (u64)(2 * G.nq + __builtin_popcount(d)) * L_ * 8ULL;
    }
    const u32 cnt = (u32)(offs.size() - first);
    if (cnt) passes.push_back(PassRange{first, cnt, bytes});
    pass.clear();
    pool_.push_back(std::move(pass));
    open_.pop_front();
    ++lo_;
  }
};

// Gate lists of at least 2 kPlanChunk ops are compiled in chunks of
// kPlanChunk ops, on helper threads: the passes of consecutive chunks,
// concatenated, apply the gates in program order (gates at the start of a
// chunk just cannot join the previous chunk's open passes, about one extra
// pass per boundary). Chunk boundaries depend on the op count only, so the
// plan does not depend on how many threads were free.
constexpr u64 kPlanChunk = 1ull << 19;
constexpr int kPlanMaxHelpers = 15;  // helper threads over all callers at once
inline std::atomic<int> g_plan_helpers{0};

inline void plan_chunked(u32 n, u32 L, const sq_op *ops, u64 count, WideBuilder &out) {
  const u64 nch = (count + kPlanChunk - 1) / kPlanChunk;
  std::vector<WideBuilder> part(nch);
  std::atomic<u64> next{0};
  auto work = [&]() {
    for (;;) {
      const u64 c = next.fetch_add(1);
      if (c >= nch) break;
      const u64 lo = c * kPlanChunk, hi = std::min<u64>(count, lo + kPlanChunk);
      WideBuilder &b = part[c];
      b.init(n, L);
      for (u64 i = lo; i < hi; ++i) b.add(ops[i].type, ops[i].q0, ops[i].q1);
      b.flush();
    }
  };
  const int hw = std::max(1, (int)std::thread::hardware_concurrency());
  const int cap = std::min(kPlanMaxHelpers, hw - 1);
  const int want = (int)std::min<u64>(nch - 1, 7);
  int got = 0;
  while (got < want) {
    int cur = g_plan_helpers.load();
    if (cur >= cap) break;
    if (g_plan_helpers.compare_exchange_weak(cur, cur + 1)) ++got;
  }
  std::vector<std::thread> helpers;
  for (int i = 0; i < got; ++i) {
    try {
      helpers.emplace_back(work);
    } catch (...) {  // no thread to be had: the others (and this one) take its chunks
      break;
    }
  }
  work();
  for (std::thread &t : helpers) t.join();
  g_plan_helpers -= got;
  out.words.clear();
  out.offs.clear();
  out.passes.clear();
  for (const WideBuilder &b : part) {
    const u32 wbase = (u32)out.words.size();
    const u64 obase = out.offs.size();
    out.words.insert(out.words.end(), b.words.begin(), b.words.end());
    for (u32 o : b.offs) out.offs.push_back(o + wbase);
    for (PassRange r : b.passes) {
      r.offset += obase;
      out.passes.push_back(r);
    }
  }
}

// The plan of a host gate list (gates only): one builder, or chunks on
// helper threads for long lists.
inline void plan_gate_list(u32 n, u32 L, const sq_op *ops, u64 count, WideBuilder &out) {
  if (count >= 2 * kPlanChunk) {
    plan_chunked(n, L, ops, count, out);
    return;
  }
  out.init(n, L);
  for (u64 i = 0; i < count; ++i) out.add(ops[i].type, ops[i].q0, ops[i].q1);
  out.flush();
}

// ============================================================== pair groups
struct HGroup {
  u32 qa, qb;
  u64 ops;
  u32 nops;
  bool alive;
};

inline u32 dirty_flags(u64 ops) {
  u32 f = 0;
  for (; ops; ops >>= 4) {
    switch ((u32)(ops & 15)) {
      case UOP_H_A: f |= GD_XA | GD_ZA; break;
      case UOP_S_A: case UOP_SDG_A: f |= GD_ZA; break;
      case UOP_H_B: f |= GD_XB | GD_ZB; break;
      case UOP_S_B: case UOP_SDG_B: f |= GD_ZB; break;
      case UOP_CX_AB: f |= GD_XB | GD_ZA; break;
      case UOP_CX_BA: f |= GD_XA | GD_ZB; break;
      case UOP_CZ: f |= GD_ZA | GD_ZB; break;
      default: break;
    }
  }
  return f;
}

inline u32 one_qubit_uop(u32 type) {
  switch (type) {
    case SQ_H: return UOP_H_A;
    case SQ_S: return UOP_S_A;
    case SQ_SDG: return UOP_SDG_A;
    case SQ_X: return UOP_X_A;
    case SQ_Y: return UOP_Y_A;
    default: return UOP_Z_A;
  }
}

class PassBuilder {
 public:
  std::vector<Group> groups;
  std::vector<PassRange> passes;

  void init(u32 n, u32 L) {
    n_ = n;
    L_ = L;
    owner_.assign(n, -1);
    epoch_of_.assign(n, 0);
    epoch_ = 1;
    groups.clear();
    passes.clear();
    cur_.clear();
  }

  void add(u32 type, u32 a, u32 b) {
    if (type == SQ_I) return;
    // CY, SWAP, iSWAP as products of the pair micro-ops, in time order
    if (type == SQ_CY) {
      add(SQ_SDG, b, 0);
      add(SQ_CX, a, b);
      add(SQ_S, b, 0);
      return;
    }
    if (type == SQ_SWAP) {
      add(SQ_CX, a, b);
      add(SQ_CX, b, a);
      add(SQ_CX, a, b);
      return;
    }
    if (type == SQ_ISWAP) {
      add(SQ_S, a, 0);
      add(SQ_S, b, 0);
      add(SQ_CZ, a, b);
      add(SQ_SWAP, a, b);
      return;
    }
    if (!is_two_qubit(type)) {
      int g = find(a);
      if (g >= 0 && cur_[g].nops >= 16) { flush(); g = -1; }
      if (g < 0) g = open(a, G_SINGLE);
      const u32 code = one_qubit_uop(type) + (cur_[g].qa == a ? 0u : 6u);
      push(g, code);
      return;
    }
    int ga = find(a), gb = find(b), g;
    if (ga >= 0 && ga == gb) {
      g = ga;
      if (cur_[g].nops >= 16) { flush(); g = open(a, b); }
    } else {
      const bool pair_a = ga >= 0 && cur_[ga].qb != G_SINGLE;
      const bool pair_b = gb >= 0 && cur_[gb].qb != G_SINGLE;
      const u32 need = (ga >= 0 ? cur_[ga].nops : 0) + (gb >= 0 ? cur_[gb].nops : 0) + 1;
      if (pair_a || pair_b || need > 16) { flush(); ga = gb = -1; }
      if (ga < 0 && gb < 0) {
        g = open(a, b);
      } else if (gb < 0) {
        g = ga;
        cur_[g].qb = b;
        bind(b, g);
      } else if (ga < 0) {
        g = gb;            // b stays slot A, a becomes slot B
        cur_[g].qb = a;
        bind(a, g);
      } else {
        g = ga;            // merge the single group of b into slot B of a's group
        cur_[g].qb = b;
        bind(b, g);
        const u64 ob = cur_[gb].ops;
        for (u32 k = 0; k < cur_[gb].nops; ++k) push(g, (u32)((ob >> (4 * k)) & 15) + 6u);
        cur_[gb].alive = false;
      }
    }
    const bool a_is_A = cur_[g].qa == a;
    push(g, type == SQ_CZ ? UOP_CZ : (a_is_A ? UOP_CX_AB : UOP_CX_BA));
  }

  void flush() {
    const u64 off = groups.size();
    u64 bytes = 0;
    for (const HGroup &h : cur_) {
      if (!h.alive || h.nops == 0) continue;
      const u32 f = dirty_flags(h.ops);
      groups.push_back(Group{h.qa | f, h.qb, h.ops});
      const u32 reads = (h.qb == G_SINGLE) ? 2 : 4;
      const u32 writes = (u32)__builtin_popcount(f);
      bytes += (u64)(reads + writes) * L_ * 8ULL;
    }
    const u32 cnt = (u32)(groups.size() - off);
    if (cnt) passes.push_back(PassRange{off, cnt, bytes});
    cur_.clear();
    if (++epoch_ == 0) {
      std::fill(epoch_of_.begin(), epoch_of_.end(), 0u);
      epoch_ = 1;
    }
  }

 private:
  u32 n_ = 0, L_ = 0, epoch_ = 1;
  std::vector<int32_t> owner_;
  std::vector<u32> epoch_of_;
  std::vector<HGroup> cur_;

  int find(u32 q) const { return epoch_of_[q] == epoch_ ? owner_[q] : -1; }
  void bind(u32 q, int g) {
    epoch_of_[q] = epoch_;
    owner_[q] = g;
  }
  int open(u32 a, u32 b) {
    cur_.push_back(HGroup{a, b, 0, 0, true});
    const int g = (int)cur_.size() - 1;
    bind(a, g);
    if (b != G_SINGLE) bind(b, g);
    return g;
  }
  void push(int g, u32 code) {
    cur_[g].ops |= (u64)code << (4 * cur_[g].nops);
    cur_[g].nops += 1;
  }
};

}  // namespace sq
