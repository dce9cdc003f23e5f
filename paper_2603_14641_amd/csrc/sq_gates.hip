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

}  // namespace sq
