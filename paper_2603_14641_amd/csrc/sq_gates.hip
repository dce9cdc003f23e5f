// Gate passes (tableau evolution): the fused group kernel and the sign reduction.
#include "sq_device.h"

namespace sq {

// ---------------------------------------------------------------------------
// a2: one fused gate pass. Each group is a short sequence of gates on one or
// two qubits; groups of a pass act on disjoint qubits, so every (group,
// row word) update is independent. The column rules (pre-gate values on the
// right-hand side) per 64 rows at once:
//   H:   r ^= x&z;  (x, z) <- (z, x)
//   S:   r ^= x&z;  z ^= x          S^dagger: r ^= x&~z; z ^= x
//   X:   r ^= z     Y: r ^= x^z     Z: r ^= x
//   CX(c,t): r ^= x_c & z_t & ~(x_t ^ z_c); x_t ^= x_c; z_c ^= z_t
//   CZ(a,b): r ^= x_a & x_b & (z_a ^ z_b);  z_a ^= x_b; z_b ^= x_a
// A thread owns WPT consecutive row words and walks the groups of its
// chunk, keeping the sign changes in registers; the per-chunk sign words go
// to sign_part and are XOR-reduced by k_sign_reduce.
template <int WPT>
__device__ __forceinline__ void run_uops(u64 ops, u64 (&xa)[WPT], u64 (&za)[WPT], u64 (&xb)[WPT], u64 (&zb)[WPT],
                                         u64 (&s)[WPT]) {
  for (; ops != 0; ops >>= 4) {
    switch ((u32)(ops & 15ULL)) {
      case UOP_H_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xa[k] & za[k]; const u64 t = xa[k]; xa[k] = za[k]; za[k] = t; }
        break;
      case UOP_S_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xa[k] & za[k]; za[k] ^= xa[k]; }
        break;
      case UOP_SDG_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xa[k] & ~za[k]; za[k] ^= xa[k]; }
        break;
      case UOP_X_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= za[k];
        break;
      case UOP_Y_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= xa[k] ^ za[k];
        break;
      case UOP_Z_A:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= xa[k];
        break;
      case UOP_H_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xb[k] & zb[k]; const u64 t = xb[k]; xb[k] = zb[k]; zb[k] = t; }
        break;
      case UOP_S_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xb[k] & zb[k]; zb[k] ^= xb[k]; }
        break;
      case UOP_SDG_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xb[k] & ~zb[k]; zb[k] ^= xb[k]; }
        break;
      case UOP_X_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= zb[k];
        break;
      case UOP_Y_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= xb[k] ^ zb[k];
        break;
      case UOP_Z_B:
#pragma unroll
        for (int k = 0; k < WPT; ++k) s[k] ^= xb[k];
        break;
      case UOP_CX_AB:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xa[k] & zb[k] & ~(xb[k] ^ za[k]); xb[k] ^= xa[k]; za[k] ^= zb[k]; }
        break;
      case UOP_CX_BA:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xb[k] & za[k] & ~(xa[k] ^ zb[k]); xa[k] ^= xb[k]; zb[k] ^= za[k]; }
        break;
      case UOP_CZ:
#pragma unroll
        for (int k = 0; k < WPT; ++k) { s[k] ^= xa[k] & xb[k] & (za[k] ^ zb[k]); const u64 ta = za[k] ^ xb[k]; zb[k] ^= xa[k]; za[k] = ta; }
        break;
      default:
        break;
    }
  }
}

template <int WPT, int B>
__global__ __launch_bounds__(1024) void k_layer(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ sign_part,
                                                 const Group *__restrict__ groups, u32 ngroups, u32 gpc, u32 Ls, u32 L) {
  const u32 w = (blockIdx.x * blockDim.x + threadIdx.x) * WPT;
  if (w >= L) return;
  const u32 g0 = blockIdx.y * gpc;
  const u32 g1 = min(g0 + gpc, ngroups);
  u64 s[WPT];
#pragma unroll
  for (int k = 0; k < WPT; ++k) s[k] = 0;

  u32 g = g0;
  for (; g + B <= g1; g += B) {
    Group G[B];
    u64 xa[B][WPT], za[B][WPT], xb[B][WPT], zb[B][WPT];
#pragma unroll
    for (int b = 0; b < B; ++b) G[b] = groups[g + b];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const size_t ca = (size_t)(G[b].q0 & GQ_MASK) * Ls + w;
      ldw<WPT>(X + ca, xa[b]);
      ldw<WPT>(Z + ca, za[b]);
      if (G[b].q1 != G_SINGLE) {
        const size_t cb = (size_t)G[b].q1 * Ls + w;
        ldw<WPT>(X + cb, xb[b]);
        ldw<WPT>(Z + cb, zb[b]);
      } else {
#pragma unroll
        for (int k = 0; k < WPT; ++k) { xb[b][k] = 0; zb[b][k] = 0; }
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      run_uops<WPT>(G[b].ops, xa[b], za[b], xb[b], zb[b], s);
      const u32 f = G[b].q0;
      const size_t ca = (size_t)(f & GQ_MASK) * Ls + w;
      if (f & GD_XA) stw<WPT>(X + ca, xa[b]);
      if (f & GD_ZA) stw<WPT>(Z + ca, za[b]);
      if (G[b].q1 != G_SINGLE) {
        const size_t cb = (size_t)G[b].q1 * Ls + w;
        if (f & GD_XB) stw<WPT>(X + cb, xb[b]);
        if (f & GD_ZB) stw<WPT>(Z + cb, zb[b]);
      }
    }
  }
  for (; g < g1; ++g) {
    const Group G = groups[g];
    u64 xa[WPT], za[WPT], xb[WPT], zb[WPT];
    const size_t ca = (size_t)(G.q0 & GQ_MASK) * Ls + w;
    ldw<WPT>(X + ca, xa);
    ldw<WPT>(Z + ca, za);
    const bool two = G.q1 != G_SINGLE;
    const size_t cb = two ? (size_t)G.q1 * Ls + w : 0;
    if (two) {
      ldw<WPT>(X + cb, xb);
      ldw<WPT>(Z + cb, zb);
    } else {
#pragma unroll
      for (int k = 0; k < WPT; ++k) { xb[k] = 0; zb[k] = 0; }
    }
    run_uops<WPT>(G.ops, xa, za, xb, zb, s);
    if (G.q0 & GD_XA) stw<WPT>(X + ca, xa);
    if (G.q0 & GD_ZA) stw<WPT>(Z + ca, za);
    if (two) {
      if (G.q0 & GD_XB) stw<WPT>(X + cb, xb);
      if (G.q0 & GD_ZB) stw<WPT>(Z + cb, zb);
    }
  }
  stw<WPT>(sign_part + (size_t)blockIdx.y * Ls + w, s);
}

__global__ void k_sign_reduce(u64 *__restrict__ R, const u64 *__restrict__ sign_part, u32 nchunks, u32 Ls, u32 L) {
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= L) return;
  u64 acc = 0;
  for (u32 c = 0; c < nchunks; ++c) acc ^= sign_part[(size_t)c * Ls + w];
  R[w] ^= acc;
}

// Launchers.
hipError_t launch_layer(const TabDev &t, const Group *groups, u32 ngroups, u32 block, u32 wpt, u32 gpc,
                        u64 *sign_part, hipStream_t s) {
  const u32 tiles = cdiv(t.L, (u64)block * wpt);
  const u32 chunks = cdiv(ngroups, gpc);
  dim3 grid(tiles, chunks);
  if (wpt == 2)
    hipLaunchKernelGGL((k_layer<2, 4>), grid, dim3(block), 0, s, t.X, t.Z, sign_part, groups, ngroups, gpc, t.Ls, t.L);
  else
    hipLaunchKernelGGL((k_layer<1, 4>), grid, dim3(block), 0, s, t.X, t.Z, sign_part, groups, ngroups, gpc, t.Ls, t.L);
  return hipGetLastError();
}

hipError_t launch_sign_reduce(const TabDev &t, const u64 *sign_part, u32 nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_reduce, dim3(cdiv(t.L, 256)), dim3(256), 0, s, t.R, sign_part, nchunks, t.Ls, t.L);
  return hipGetLastError();
}

}  // namespace sq
