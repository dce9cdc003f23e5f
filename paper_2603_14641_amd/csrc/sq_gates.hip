// Gate passes (tableau evolution): the fused group kernel and the sign reduction.
#include "sq_device.h"

namespace sq {

// ---------------------------------------------------------------------------
// a2: one fused gate pass. Each group is a short gate sequence on up to
// WG_MAXQ qubits; groups of a pass act on disjoint qubits, so every (group,
// row word) update is independent. The column rules (pre-gate values on the
// right-hand side) per 64 rows at once:
//   H:   r ^= x&z;  (x, z) <- (z, x)
//   S:   r ^= x&z;  z ^= x          S^dagger: r ^= x&~z; z ^= x
//   X:   r ^= z     Y: r ^= x^z     Z: r ^= x
//   CX(c,t): r ^= x_c & z_t & ~(x_t ^ z_c); x_t ^= x_c; z_c ^= z_t
//   CZ(a,b): r ^= x_a & x_b & (z_a ^ z_b);  z_a ^= x_b; z_b ^= x_a
//   SWAP(a,b): exchange the two columns (sign unchanged)
// (CY and iSWAP arrive as products of these.)
// A thread owns WPT consecutive row words. For each group of its chunk it
// loads the group's columns into registers, runs the micro-ops (their slots
// are uniform over the wave, so the dispatch below is a scalar branch and
// every register index is a constant), and stores the changed columns. Sign
// changes stay in registers for the whole chunk; the per-chunk sign words go
// to sign_part and are XOR-reduced by k_sign_reduce.
template <int WPT>
struct Cols {
  u64 x[WG_MAXQ][WPT], z[WG_MAXQ][WPT];
};

template <int A, int WPT>
__device__ __forceinline__ void op1(u32 t, Cols<WPT> &c, u64 (&s)[WPT]) {
#pragma unroll
  for (int k = 0; k < WPT; ++k) {
    u64 &x = c.x[A][k], &z = c.z[A][k];
    switch (t) {
      case WOP_H: { s[k] ^= x & z; const u64 v = x; x = z; z = v; } break;
      case WOP_S: s[k] ^= x & z; z ^= x; break;
      case WOP_SDG: s[k] ^= x & ~z; z ^= x; break;
      case WOP_X: s[k] ^= z; break;
      case WOP_Y: s[k] ^= x ^ z; break;
      default: s[k] ^= x; break;  // Z
    }
  }
}

template <int A, int B, int WPT>
__device__ __forceinline__ void op2(u32 t, Cols<WPT> &c, u64 (&s)[WPT]) {
  if constexpr (A != B) {
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      u64 &xa = c.x[A][k], &za = c.z[A][k], &xb = c.x[B][k], &zb = c.z[B][k];
      if (t == WOP_CX) {
        s[k] ^= xa & zb & ~(xb ^ za);
        xb ^= xa;
        za ^= zb;
      } else if (t == WOP_SWAP) {
        const u64 tx = xa, tz = za;
        xa = xb;
        za = zb;
        xb = tx;
        zb = tz;
      } else {
        s[k] ^= xa & xb & (za ^ zb);
        const u64 ta = za ^ xb;
        zb ^= xa;
        za = ta;
      }
    }
  }
}

template <int A, int WPT>
__device__ __forceinline__ void op2_row(u32 t, u32 b, Cols<WPT> &c, u64 (&s)[WPT]) {
  switch (b) {
    case 0: op2<A, 0>(t, c, s); break;
    case 1: op2<A, 1>(t, c, s); break;
    case 2: op2<A, 2>(t, c, s); break;
    case 3: op2<A, 3>(t, c, s); break;
    case 4: op2<A, 4>(t, c, s); break;
    case 5: op2<A, 5>(t, c, s); break;
    case 6: op2<A, 6>(t, c, s); break;
    default: op2<A, 7>(t, c, s); break;
  }
}

template <int WPT>
__device__ __forceinline__ void run_op(u32 op, Cols<WPT> &c, u64 (&s)[WPT]) {
  static_assert(WG_MAXQ == 8, "the slot dispatch below covers 8 slots");
  const u32 t = op & 15u, a = (op >> 4) & 15u, b = (op >> 8) & 15u;
  if (t < WOP_CX) {
    switch (a) {
      case 0: op1<0>(t, c, s); break;
      case 1: op1<1>(t, c, s); break;
      case 2: op1<2>(t, c, s); break;
      case 3: op1<3>(t, c, s); break;
      case 4: op1<4>(t, c, s); break;
      case 5: op1<5>(t, c, s); break;
      case 6: op1<6>(t, c, s); break;
      default: op1<7>(t, c, s); break;
    }
  } else {
    switch (a) {
      case 0: op2_row<0>(t, b, c, s); break;
      case 1: op2_row<1>(t, b, c, s); break;
      case 2: op2_row<2>(t, b, c, s); break;
      case 3: op2_row<3>(t, b, c, s); break;
      case 4: op2_row<4>(t, b, c, s); break;
      case 5: op2_row<5>(t, b, c, s); break;
      case 6: op2_row<6>(t, b, c, s); break;
      default: op2_row<7>(t, b, c, s); break;
    }
  }
}

template <int WPT>
__device__ __forceinline__ void load_group(const u32 *rec, const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                           u32 Ls, u32 w, Cols<WPT> &c) {
  const u32 nq = rec[0] & 15u;
#pragma unroll
  for (u32 i = 0; i < WG_MAXQ; ++i) {
    if (i < nq) {
      const size_t o = (size_t)rec[1 + i] * Ls + w;
      ldw_nt<WPT>(X + o, c.x[i]);
      ldw_nt<WPT>(Z + o, c.z[i]);
    }
  }
}

template <int WPT>
__device__ __forceinline__ void finish_group(const u32 *rec, u64 *__restrict__ X, u64 *__restrict__ Z, u32 Ls, u32 w,
                                             Cols<WPT> &c, u64 (&s)[WPT]) {
  const u32 hdr = rec[0];
  const u32 nq = hdr & 15u, nops = (hdr >> WH_NOPS_SHIFT) & 63u;
  const u32 *ops = rec + 1 + nq;
  // two micro-ops per word; the next word's scalar load is issued before
  // the current word's ops run, so its latency is hidden
  const u32 nw = (nops + 1u) >> 1;
  u32 cur = ops[0];
  for (u32 i = 0; i < nw; ++i) {
    const u32 nxt = (i + 1 < nw) ? ops[i + 1] : 0u;
    run_op<WPT>(cur & 0xFFFFu, c, s);
    if (2 * i + 1 < nops) run_op<WPT>(cur >> 16, c, s);
    cur = nxt;
  }
#pragma unroll
  for (u32 i = 0; i < WG_MAXQ; ++i) {
    if (i < nq) {
      const size_t o = (size_t)rec[1 + i] * Ls + w;
      if ((hdr >> (WH_DX_SHIFT + i)) & 1u) stw_nt<WPT>(X + o, c.x[i]);
      if ((hdr >> (WH_DZ_SHIFT + i)) & 1u) stw_nt<WPT>(Z + o, c.z[i]);
    }
  }
}

// B groups are loaded before the first is computed, so a wave keeps the
// columns of B groups in flight (B = 1 in use: with B = 2 the compiler moves
// the column arrays to scratch memory).
template <int WPT, int B>
__global__ __launch_bounds__(512) void k_layer(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ sign_part,
                                                const u32 *__restrict__ words, const u32 *__restrict__ offs,
                                                u32 ngroups, u32 gpc, u32 Ls, u32 L) {
  const u32 w = (blockIdx.x * blockDim.x + threadIdx.x) * WPT;
  if (w >= L) return;
  const u32 g0 = blockIdx.y * gpc;
  const u32 g1 = min(g0 + gpc, ngroups);
  u64 s[WPT];
#pragma unroll
  for (int k = 0; k < WPT; ++k) s[k] = 0;
  Cols<WPT> c[B];
  for (u32 g = g0; g < g1; g += B) {
    const u32 *rec[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      rec[b] = g + b < g1 ? words + offs[g + b] : nullptr;
      if (rec[b]) load_group<WPT>(rec[b], X, Z, Ls, w, c[b]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (rec[b]) finish_group<WPT>(rec[b], X, Z, Ls, w, c[b], s);
  }
  stw<WPT>(sign_part + (size_t)blockIdx.y * Ls + w, s);
}

// Grid (row tiles, slices): slice y XORs the partials of chunks y, y + S,
// y + 2S, ... and folds them into R with one 64-bit atomic XOR (the order of
// the XORs does not matter).
__global__ void k_sign_reduce(u64 *__restrict__ R, const u64 *__restrict__ sign_part, u32 nchunks, u32 Ls, u32 L) {
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= L) return;
  u64 acc = 0;
  for (u32 c = blockIdx.y; c < nchunks; c += gridDim.y) acc ^= sign_part[(size_t)c * Ls + w];
  if (acc) atomicXor(&R[w], acc);
}

// Launchers.
hipError_t launch_layer(const TabDev &t, const u32 *words, const u32 *offs, u32 ngroups, u32 block, u32 wpt,
                        u32 gpc, u64 *sign_part, hipStream_t s) {
  const u32 tiles = cdiv(t.L, (u64)block * wpt);
  const u32 chunks = cdiv(ngroups, gpc);
  dim3 grid(tiles, chunks);
  if (wpt == 2)
    hipLaunchKernelGGL((k_layer<2, 1>), grid, dim3(block), 0, s, t.X, t.Z, sign_part, words, offs, ngroups, gpc, t.Ls,
                       t.L);
  else
    hipLaunchKernelGGL((k_layer<1, 1>), grid, dim3(block), 0, s, t.X, t.Z, sign_part, words, offs, ngroups, gpc, t.Ls,
                       t.L);
  return hipGetLastError();
}

hipError_t launch_sign_reduce(const TabDev &t, const u64 *sign_part, u32 nchunks, hipStream_t s) {
  const u32 slices = std::min<u32>(std::max<u32>(nchunks, 1), 64);
  hipLaunchKernelGGL(k_sign_reduce, dim3(cdiv(t.L, 256), slices), dim3(256), 0, s, t.R, sign_part, nchunks, t.Ls,
                     t.L);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operator-tableau gate pass (the tableau of Algorithm alg:stim: for each
// qubit q the images A_q of X_q and B_q of Z_q over generator positions k,
// a sign per image). Its bits are those of the state tableau, position k
// being row pair (D_k, S_k): B_q has x part x_q(S_k) and z part x_q(D_k),
// A_q has x part z_q(S_k) and z part z_q(D_k). Appending a gate therefore
// moves bits exactly like the column rules above; what differs is the signs,
// one per image, which change by the phase of products of whole images:
//   H: swap A_q, B_q             S: A_q <- -i A_q B_q    S^dagger: A_q <- i A_q B_q
//   X: -B_q   Z: -A_q   Y: both  CX(c,t): A_c <- A_c A_t, B_t <- B_t B_c
//   CZ(a,b): A_a <- A_a B_b, A_b <- A_b B_a     SWAP: swap the images
// The phase of P Q over 64 positions, with Y = iXZ, is (mod 4)
//   |P.x & P.z| + |Q.x & Q.z| + 2 |P.z & Q.x| - |(P.x ^ Q.x) & (P.z ^ Q.z)|,
// the sum of Aaronson and Gottesman's g function over the positions.
// A workgroup takes one group at a time and walks every position word of its
// columns (thread = position word: the D word w and the S word K + w of each
// column), so each product's phase is a reduction within the workgroup; a
// micro-op's two products are bit-sliced 2-bit counters 2i and 2i + 1 of a
// 64-bit pair. Thread 0 then replays the group's micro-ops on the 2 sign
// bits per qubit (held in R: word q/64 the A signs, word K + q/64 the B
// signs) and XORs the changes in; the groups of a pass touch disjoint qubits.
__device__ __forceinline__ u32 prod_phase(u64 px, u64 pz, u64 qx, u64 qz) {
  return ((u32)__popcll(px & pz) + (u32)__popcll(qx & qz) + 2u * (u32)__popcll(pz & qx) -
          (u32)__popcll((px ^ qx) & (pz ^ qz))) & 3u;
}

// the phases a micro-op's products pick up, c1 | c2 << 2, from pre-op values
template <int A>
__device__ __forceinline__ u32 ph1(const Cols<2> &c) {
  return prod_phase(c.z[A][1], c.z[A][0], c.x[A][1], c.x[A][0]);  // A_a B_a
}

template <int A, int B>
__device__ __forceinline__ u32 ph2(u32 t, const Cols<2> &c) {
  if constexpr (A == B) {
    return 0u;
  } else {
    if (t == WOP_CX)  // A_a A_b, B_b B_a
      return prod_phase(c.z[A][1], c.z[A][0], c.z[B][1], c.z[B][0]) |
             (prod_phase(c.x[B][1], c.x[B][0], c.x[A][1], c.x[A][0]) << 2);
    if (t == WOP_CZ)  // A_a B_b, A_b B_a
      return prod_phase(c.z[A][1], c.z[A][0], c.x[B][1], c.x[B][0]) |
             (prod_phase(c.z[B][1], c.z[B][0], c.x[A][1], c.x[A][0]) << 2);
    return 0u;  // SWAP
  }
}

template <int A>
__device__ __forceinline__ u32 ph2_row(u32 t, u32 b, const Cols<2> &c) {
  switch (b) {
    case 0: return ph2<A, 0>(t, c);
    case 1: return ph2<A, 1>(t, c);
    case 2: return ph2<A, 2>(t, c);
    case 3: return ph2<A, 3>(t, c);
    case 4: return ph2<A, 4>(t, c);
    case 5: return ph2<A, 5>(t, c);
    case 6: return ph2<A, 6>(t, c);
    default: return ph2<A, 7>(t, c);
  }
}

__device__ __forceinline__ u32 op_phase(u32 op, const Cols<2> &c) {
  const u32 t = op & 15u, a = (op >> 4) & 15u, b = (op >> 8) & 15u;
  if (t == WOP_S || t == WOP_SDG) {
    switch (a) {
      case 0: return ph1<0>(c);
      case 1: return ph1<1>(c);
      case 2: return ph1<2>(c);
      case 3: return ph1<3>(c);
      case 4: return ph1<4>(c);
      case 5: return ph1<5>(c);
      case 6: return ph1<6>(c);
      default: return ph1<7>(c);
    }
  }
  if (t < WOP_CX) return 0u;
  switch (a) {
    case 0: return ph2_row<0>(t, b, c);
    case 1: return ph2_row<1>(t, b, c);
    case 2: return ph2_row<2>(t, b, c);
    case 3: return ph2_row<3>(t, b, c);
    case 4: return ph2_row<4>(t, b, c);
    case 5: return ph2_row<5>(t, b, c);
    case 6: return ph2_row<6>(t, b, c);
    default: return ph2_row<7>(t, b, c);
  }
}

// (lo, hi) += (nlo, nhi): 64 independent 2-bit counters, bit-sliced
__device__ __forceinline__ void add2(u64 &lo, u64 &hi, u64 nlo, u64 nhi) {
  hi ^= nhi ^ (lo & nlo);
  lo ^= nlo;
}

// Replay a group's micro-ops on its qubits' image signs, given the total
// phase counters (lo, hi) of its products. The phase exponent of every
// product must be even; an odd one sets flag bit 0.
__device__ void replay_signs(const u32 *rec, u64 lo, u64 hi, u64 *__restrict__ R, u32 K, u32 *__restrict__ flags) {
  const u32 hdr = rec[0];
  const u32 nq = hdr & 15u, nops = (hdr >> WH_NOPS_SHIFT) & 63u;
  const u32 *ops = rec + 1 + nq;
  u32 sa[WG_MAXQ], sb[WG_MAXQ], sa0[WG_MAXQ], sb0[WG_MAXQ];  // signs of A_q and B_q per slot
  for (u32 i = 0; i < nq; ++i) {
    const u32 q = rec[1 + i];
    sa[i] = sa0[i] = (u32)(R[q >> 6] >> (q & 63u)) & 1u;
    sb[i] = sb0[i] = (u32)(R[K + (q >> 6)] >> (q & 63u)) & 1u;
  }
  u32 odd = 0;
  for (u32 k = 0; k < nops; ++k) {
    const u32 op = (ops[k >> 1] >> ((k & 1u) * 16u)) & 0xFFFFu;
    const u32 t = op & 15u, a = (op >> 4) & 15u, b = (op >> 8) & 15u;
    const u32 c1 = (u32)((lo >> (2 * k)) & 1u) | ((u32)((hi >> (2 * k)) & 1u) << 1);
    const u32 c2 = (u32)((lo >> (2 * k + 1)) & 1u) | ((u32)((hi >> (2 * k + 1)) & 1u) << 1);
    u32 e1, e2;
    switch (t) {
      case WOP_H: { const u32 v = sa[a]; sa[a] = sb[a]; sb[a] = v; } break;
      case WOP_S: e1 = (2 * sa[a] + 2 * sb[a] + 3 + c1) & 3u; odd |= e1; sa[a] = e1 >> 1; break;
      case WOP_SDG: e1 = (2 * sa[a] + 2 * sb[a] + 1 + c1) & 3u; odd |= e1; sa[a] = e1 >> 1; break;
      case WOP_X: sb[a] ^= 1u; break;
      case WOP_Y: sa[a] ^= 1u; sb[a] ^= 1u; break;
      case WOP_Z: sa[a] ^= 1u; break;
      case WOP_CX:
        e1 = (2 * sa[a] + 2 * sa[b] + c1) & 3u;
        e2 = (2 * sb[b] + 2 * sb[a] + c2) & 3u;
        odd |= e1 | e2;
        sa[a] = e1 >> 1;
        sb[b] = e2 >> 1;
        break;
      case WOP_CZ:
        e1 = (2 * sa[a] + 2 * sb[b] + c1) & 3u;
        e2 = (2 * sa[b] + 2 * sb[a] + c2) & 3u;
        odd |= e1 | e2;
        sa[a] = e1 >> 1;
        sa[b] = e2 >> 1;
        break;
      default: {  // SWAP
        u32 v = sa[a]; sa[a] = sa[b]; sa[b] = v;
        v = sb[a]; sb[a] = sb[b]; sb[b] = v;
      } break;
    }
  }
  if (odd & 1u) atomicOr(flags, 1u);
  for (u32 i = 0; i < nq; ++i) {
    const u32 q = rec[1 + i];
    if (sa0[i] != sa[i]) atomicXor(&R[q >> 6], 1ULL << (q & 63u));
    if (sb0[i] != sb[i]) atomicXor(&R[K + (q >> 6)], 1ULL << (q & 63u));
  }
}

// Grid (position tiles, group chunks), as k_layer: a thread owns position
// word w (destabilizer word w and stabilizer word K + w of each column of
// the group) and walks its chunk's groups, applying the micro-ops and adding
// each product's phase over its 64 positions into bit-sliced counters. Per
// group a wave sums its counters (butterfly) and lane 0 writes them to
// part[(g - g_base) * nw + wave], nw being the waves along the position
// dimension; k_layer_op_signs then adds a group's nw partials and replays
// its micro-ops on the signs. No barriers: every lane takes part in the
// butterflies (lanes past the last position word hold zero counters).
__global__ __launch_bounds__(256) void k_layer_op(u64 *__restrict__ X, u64 *__restrict__ Z,
                                                  const u32 *__restrict__ words, const u32 *__restrict__ offs,
                                                  u32 g_base, u32 g_end, u32 gpc, u32 Ls, u32 K,
                                                  u64x2 *__restrict__ part) {
  const u32 tid = threadIdx.x, lane = tid & 63u;
  const u32 w = blockIdx.x * blockDim.x + tid;
  const bool act = w < K;
  const u32 nw = gridDim.x * (blockDim.x >> 6), wv = blockIdx.x * (blockDim.x >> 6) + (tid >> 6);
  const u32 g0 = g_base + blockIdx.y * gpc;
  const u32 g1 = min(g0 + gpc, g_end);
  u64 sdummy[2];
  for (u32 g = g0; g < g1; ++g) {
    const u32 *rec = words + offs[g];
    const u32 hdr = rec[0];
    const u32 nq = hdr & 15u, nops = (hdr >> WH_NOPS_SHIFT) & 63u;
    const u32 *ops = rec + 1 + nq;
    Cols<2> c;
#pragma unroll
    for (u32 i = 0; i < WG_MAXQ; ++i) {
      c.x[i][0] = c.x[i][1] = c.z[i][0] = c.z[i][1] = 0;
      if (i < nq && act) {
        const size_t o = (size_t)rec[1 + i] * Ls + w;
        c.x[i][0] = __builtin_nontemporal_load(X + o);
        c.x[i][1] = __builtin_nontemporal_load(X + o + K);
        c.z[i][0] = __builtin_nontemporal_load(Z + o);
        c.z[i][1] = __builtin_nontemporal_load(Z + o + K);
      }
    }
    u64 lo = 0, hi = 0;
    const u32 nwd = (nops + 1u) >> 1;
    u32 cur = ops[0];
    for (u32 j = 0; j < nwd; ++j) {
      const u32 nxt = (j + 1 < nwd) ? ops[j + 1] : 0u;
#pragma unroll
      for (u32 h = 0; h < 2; ++h) {
        const u32 k = 2 * j + h;
        if (k < nops) {
          const u32 op = (cur >> (16u * h)) & 0xFFFFu;
          const u32 ph = op_phase(op, c);
          lo |= ((u64)(ph & 1u) << (2 * k)) | ((u64)((ph >> 2) & 1u) << (2 * k + 1));
          hi |= ((u64)((ph >> 1) & 1u) << (2 * k)) | ((u64)((ph >> 3) & 1u) << (2 * k + 1));
          run_op<2>(op, c, sdummy);
        }
      }
      cur = nxt;
    }
    if (act) {
#pragma unroll
      for (u32 i = 0; i < WG_MAXQ; ++i) {
        if (i < nq) {
          const size_t o = (size_t)rec[1 + i] * Ls + w;
          if ((hdr >> (WH_DX_SHIFT + i)) & 1u) {
            __builtin_nontemporal_store(c.x[i][0], X + o);
            __builtin_nontemporal_store(c.x[i][1], X + o + K);
          }
          if ((hdr >> (WH_DZ_SHIFT + i)) & 1u) {
            __builtin_nontemporal_store(c.z[i][0], Z + o);
            __builtin_nontemporal_store(c.z[i][1], Z + o + K);
          }
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) add2(lo, hi, shfl_xor_u64(lo, off), shfl_xor_u64(hi, off));
    if (lane == 0) {
      u64x2 v;
      v.x = lo;
      v.y = hi;
      part[(size_t)(g - g_base) * nw + wv] = v;
    }
  }
}

// A thread per group of [g_base, g_end): the sum of its nw partial counters,
// then the sign replay.
__global__ void k_layer_op_signs(u64 *__restrict__ R, const u32 *__restrict__ words, const u32 *__restrict__ offs,
                                 u32 g_base, u32 g_end, u32 nw, u32 K, const u64x2 *__restrict__ part,
                                 u32 *__restrict__ flags) {
  const u32 g = g_base + blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= g_end) return;
  u64 lo = 0, hi = 0;
  const u64x2 *pp = part + (size_t)(g - g_base) * nw;
  for (u32 v = 0; v < nw; ++v) {
    const u64x2 t = pp[v];
    add2(lo, hi, t.x, t.y);
  }
  replay_signs(words + offs[g], lo, hi, R, K, flags);
}

// A pass in ranges of at most max_groups groups (the partial counters of
// one range fill `part`): per range the gate kernel, then the sign replay.
hipError_t launch_layer_op(const TabDev &t, const u32 *words, const u32 *offs, u32 ngroups, u32 block, u32 gpc,
                           u32 max_groups, u64 *part, u32 *flags, hipStream_t s) {
  const u32 tiles = cdiv(t.K, block);
  const u32 nw = tiles * (block / 64);
  for (u32 g0 = 0; g0 < ngroups; g0 += max_groups) {
    const u32 g1 = std::min(ngroups, g0 + max_groups);
    hipLaunchKernelGGL(k_layer_op, dim3(tiles, cdiv(g1 - g0, gpc)), dim3(block), 0, s, t.X, t.Z, words, offs, g0, g1,
                       gpc, t.Ls, t.K, reinterpret_cast<u64x2 *>(part));
    hipLaunchKernelGGL(k_layer_op_signs, dim3(cdiv(g1 - g0, 256)), dim3(256), 0, s, t.R, words, offs, g0, g1, nw,
                       t.K, reinterpret_cast<const u64x2 *>(part), flags);
  }
  return hipGetLastError();
}

}  // namespace sq
