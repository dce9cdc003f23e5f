// HIP kernels for gfx950 (CDNA4, wave64) of the stabilizer-tableau library.
//
// All arithmetic is GF(2) bit work on 64-bit words (64 tableau rows per
// word), plus small integer phase counts; nothing here uses MFMA. Every hot
// kernel streams coalesced 64-bit column words: consecutive lanes own
// consecutive row words of one column.
#include <algorithm>

#include "sq_internal.h"

namespace sq {

typedef u64 u64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): 10 rounds, each
// multiplying counter words 0 and 2 by two odd constants and folding the
// high halves into words 1 and 3 with the round key; the key advances by two
// Weyl constants between rounds.
__device__ __forceinline__ u64 philox_word0(u64 c0, u64 c1, u64 c2, u64 c3, u64 k0, u64 k1) {
  constexpr u64 M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr u64 W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const u64 hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const u64 hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const u64 n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return c0;
}

// Coin of measurement m of shot `shot`: bit 0 of output word 0, counter (m,0,0,0), key (seed, shot).
__device__ __forceinline__ u32 coin_bit(u64 seed, u64 shot, u64 m) {
  return (u32)(philox_word0(m, 0, 0, 0, seed, shot) & 1ULL);
}

__device__ __forceinline__ u64 lanemask_lt() {
  const u32 lane = threadIdx.x & 63u;
  return (lane == 0) ? 0ULL : ((~0ULL) >> (64u - lane));
}

template <int WPT>
__device__ __forceinline__ void ldw(const u64 *p, u64 (&v)[WPT]) {
  if constexpr (WPT == 2) {
    const u64x2 t = *reinterpret_cast<const u64x2 *>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = *p;
  }
}

template <int WPT>
__device__ __forceinline__ void stw(u64 *p, const u64 (&v)[WPT]) {
  if constexpr (WPT == 2) {
    u64x2 t;
    t.x = v[0];
    t.y = v[1];
    *reinterpret_cast<u64x2 *>(p) = t;
  } else {
    *p = v[0];
  }
}

// ---------------------------------------------------------------------------
// a1: |0...0> -- zero everything, then D_i = +X_i and S_i = +Z_i.
__global__ void k_fill_zero(u64 *__restrict__ p, size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

__global__ void k_init_diag(u64 *__restrict__ X, u64 *__restrict__ Z, u32 n, u32 K, u32 Ls) {
  const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const u64 b = 1ULL << (i & 63u);
  X[(size_t)i * Ls + (i >> 6)] = b;          // D_i = X_i: column i, destabilizer word i/64
  Z[(size_t)i * Ls + K + (i >> 6)] = b;      // S_i = Z_i: column i, stabilizer word i/64
}

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

// ---------------------------------------------------------------------------
// a3: pivot search for measuring qubit q. p = the smallest stabilizer index
// with x(S_p)_q = 1 (first set bit of the stabilizer half of X column q), or
// -1. Also snapshots column q into `mask` (the rows the rowsum pass must
// touch), with the bits of D_p and S_p cleared, because the pass rewrites
// column q in place. One workgroup; thread 0 also draws the coin.
__global__ __launch_bounds__(1024) void k_pivot(const u64 *__restrict__ X, u32 Ls, u32 K, u32 L, u32 q,
                                                MeasState *__restrict__ st, u64 *__restrict__ mask, u64 seed,
                                                u64 shot, u64 m, uint8_t *__restrict__ out_bits,
                                                uint8_t *__restrict__ out_rand) {
  __shared__ u32 s_min;
  const u32 tid = threadIdx.x;
  if (tid == 0) s_min = 0xFFFFFFFFu;
  __syncthreads();
  const u64 *col = X + (size_t)q * Ls;
  u32 first = 0xFFFFFFFFu;
  for (u32 w = tid; w < K; w += blockDim.x) {
    if (col[K + w] != 0) { first = w; break; }
  }
  // wave minimum, then one LDS atomic per wave
  for (int off = 32; off > 0; off >>= 1) first = min(first, (u32)__shfl_xor((int)first, off));
  if ((tid & 63u) == 0 && first != 0xFFFFFFFFu) atomicMin(&s_min, first);
  __syncthreads();
  const u32 wmin = s_min;
  int32_t p = -1;
  if (wmin != 0xFFFFFFFFu) p = (int32_t)(wmin * 64u + (u32)__builtin_ctzll(col[K + wmin]));
  const u32 wd = (p >= 0) ? ((u32)p >> 6) : 0xFFFFFFFFu;
  const u64 bit = (p >= 0) ? (1ULL << ((u32)p & 63u)) : 0ULL;
  __shared__ u32 s_mw, s_aw;
  if (tid == 0) { s_mw = 0; s_aw = 0; }
  __syncthreads();
  u32 mw = 0, aw = 0;
  for (u32 w = tid; w < L; w += blockDim.x) {
    u64 v = col[w];
    if (w == wd || w == K + wd) v &= ~bit;
    mask[w] = v;
    mw += (v != 0);
    aw += (v != 0 && w < K);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mw += (u32)__shfl_xor((int)mw, off);
    aw += (u32)__shfl_xor((int)aw, off);
  }
  if ((tid & 63u) == 0) { atomicAdd(&s_mw, mw); atomicAdd(&s_aw, aw); }
  __syncthreads();
  if (tid == 0) {
    const u32 c = coin_bit(seed, shot, m);
    st->p = p;
    st->ncols = 0;
    st->nx = 0;
    st->nz = 0;
    st->mwords = s_mw;
    st->awords = s_aw;
    st->det_acc = 0;
    st->coin = c;
    out_rand[0] = (uint8_t)(p >= 0);
    if (p >= 0) out_bits[0] = (uint8_t)c;
  }
}

// a4: gather the pivot row S_p across all columns (one 8-byte read per column),
// pack it with wave ballots into pivx/pivz (bit j of word j/64), and compact
// the columns where S_p is not the identity into `cols`
// (entry = j | x_pj << 31 | z_pj << 30; order across waves is arbitrary).
__global__ void k_gather(const u64 *__restrict__ X, const u64 *__restrict__ Z, const u64 *__restrict__ R, u32 Ls,
                         u32 K, u32 n, MeasState *__restrict__ st, u64 *__restrict__ pivx, u64 *__restrict__ pivz,
                         u32 *__restrict__ cols) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 ws = K + ((u32)p >> 6), sh = (u32)p & 63u;
  u32 xb = 0, zb = 0;
  if (j < n) {
    xb = (u32)(X[(size_t)j * Ls + ws] >> sh) & 1u;
    zb = (u32)(Z[(size_t)j * Ls + ws] >> sh) & 1u;
  }
  const u64 bx = __ballot(xb), bz = __ballot(zb);
  const u64 nz = bx | bz;
  const u32 lane = threadIdx.x & 63u;
  u32 base = 0;
  if (lane == 0) {
    if (j < n) { pivx[j >> 6] = bx; pivz[j >> 6] = bz; }
    if (nz) base = atomicAdd(&st->ncols, (u32)__popcll(nz));
    if (bx) atomicAdd(&st->nx, (u32)__popcll(bx));
    if (bz) atomicAdd(&st->nz, (u32)__popcll(bz));
  }
  base = (u32)__shfl((int)base, 0);
  if (xb | zb) cols[base + (u32)__popcll(nz & lanemask_lt())] = j | (xb << 31) | (zb << 30);
  if (j == 0) st->rp = (u32)(R[ws] >> sh) & 1u;
}

// a5: random-case rowsum pass. For every masked row h (x_hq = 1, h not D_p or
// S_p): row_h <- S_p * row_h. Per non-identity pivot column j with Pauli P1
// = (x_pj, z_pj): x_h ^= x_pj, z_h ^= z_pj, and the phase exponent
// g(P1, P_hj) in {-1, 0, +1} is added to a bit-sliced 2-bit counter per row
// (a0 = bit 0, a1 = bit 1). g is +1 for (X,Y), (Y,Z), (Z,X) and -1 for
// (X,Z), (Y,X), (Z,Y). Counters of each column chunk go to cnt0/cnt1.
template <int WPT, int B>
__global__ __launch_bounds__(1024) void k_rowsum(u64 *__restrict__ X, u64 *__restrict__ Z,
                                                  const u64 *__restrict__ mask, const u32 *__restrict__ cols,
                                                  const MeasState *__restrict__ st, u64 *__restrict__ cnt0,
                                                  u64 *__restrict__ cnt1, u32 Ls, u32 L, u32 cpc) {
  if (st->p < 0) return;
  const u32 ncols = st->ncols;
  const u32 c0 = blockIdx.y * cpc;
  if (c0 >= ncols) return;
  const u32 c1 = min(c0 + cpc, ncols);
  const u32 w = (blockIdx.x * blockDim.x + threadIdx.x) * WPT;
  if (w >= L) return;
  u64 m[WPT];
  ldw<WPT>(mask + w, m);
  u64 any = 0;
#pragma unroll
  for (int k = 0; k < WPT; ++k) any |= m[k];
  if (any == 0) return;
  u64 a0[WPT], a1[WPT];
#pragma unroll
  for (int k = 0; k < WPT; ++k) { a0[k] = 0; a1[k] = 0; }

  auto step = [&](u32 e, const u64 (&x)[WPT], const u64 (&z)[WPT]) {
    const bool px = (e >> 31) != 0, pz = ((e >> 30) & 1u) != 0;
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      u64 plus, minus;
      if (px && !pz) { plus = x[k] & z[k]; minus = ~x[k] & z[k]; }       // P1 = X
      else if (px) { plus = ~x[k] & z[k]; minus = x[k] & ~z[k]; }        // P1 = Y
      else { plus = x[k] & ~z[k]; minus = x[k] & z[k]; }                 // P1 = Z
      plus &= m[k];
      minus &= m[k];
      a1[k] ^= a0[k] & plus;   // +1
      a0[k] ^= plus;
      a0[k] ^= minus;          // -1
      a1[k] ^= a0[k] & minus;
    }
  };

  u32 c = c0;
  for (; c + B <= c1; c += B) {
    u32 e[B];
    u64 x[B][WPT], z[B][WPT];
#pragma unroll
    for (int b = 0; b < B; ++b) e[b] = cols[c + b];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const size_t o = (size_t)(e[b] & 0x3FFFFFFFu) * Ls + w;
      ldw<WPT>(X + o, x[b]);
      ldw<WPT>(Z + o, z[b]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      step(e[b], x[b], z[b]);
      const size_t o = (size_t)(e[b] & 0x3FFFFFFFu) * Ls + w;
      if (e[b] >> 31) {
        u64 v[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) v[k] = x[b][k] ^ m[k];
        stw<WPT>(X + o, v);
      }
      if ((e[b] >> 30) & 1u) {
        u64 v[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) v[k] = z[b][k] ^ m[k];
        stw<WPT>(Z + o, v);
      }
    }
  }
  for (; c < c1; ++c) {
    const u32 e = cols[c];
    u64 x[WPT], z[WPT];
    const size_t o = (size_t)(e & 0x3FFFFFFFu) * Ls + w;
    ldw<WPT>(X + o, x);
    ldw<WPT>(Z + o, z);
    step(e, x, z);
    if (e >> 31) {
      u64 v[WPT];
#pragma unroll
      for (int k = 0; k < WPT; ++k) v[k] = x[k] ^ m[k];
      stw<WPT>(X + o, v);
    }
    if ((e >> 30) & 1u) {
      u64 v[WPT];
#pragma unroll
      for (int k = 0; k < WPT; ++k) v[k] = z[k] ^ m[k];
      stw<WPT>(Z + o, v);
    }
  }
  stw<WPT>(cnt0 + (size_t)blockIdx.y * Ls + w, a0);
  stw<WPT>(cnt1 + (size_t)blockIdx.y * Ls + w, a1);
}

// a5 (end): add the chunk counters (mod 4) of every masked row; the total
// exponent e = 2 r_h + 2 r_p + sum g must be even, and r_h <- e / 2, i.e.
// r_h ^= r_p ^ bit1(sum g). Then D_p <- old S_p (bits from pivx/pivz, sign
// r_p) and S_p <- (-1)^coin Z_q. Threads below L handle sign words, threads
// below n handle the D_p / S_p bits of one column each.
__global__ void k_finalize(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ R,
                           const u64 *__restrict__ mask, const u64 *__restrict__ pivx, const u64 *__restrict__ pivz,
                           const u64 *__restrict__ cnt0, const u64 *__restrict__ cnt1, MeasState *__restrict__ st,
                           MeasStats *__restrict__ stats, u32 Ls, u32 L, u32 K, u32 n, u32 q, u32 cpc) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    // Algorithmic bytes of this rowsum: every touched row word reads x and z
    // of each non-identity pivot column and writes x (if x_pj) and z (if z_pj).
    stats->n_random += 1;
    stats->rowsum_bytes += (u64)st->mwords * 8ULL * (2ULL * st->ncols + st->nx + st->nz);
  }
  const u32 wd = (u32)p >> 6, ws = K + wd;
  const u64 bit = 1ULL << ((u32)p & 63u);
  const u32 rp = st->rp;
  if (tid < L) {
    const u32 w = tid;
    const u64 m = mask[w];
    if (m != 0 || w == wd || w == ws) {
      u64 r = R[w];
      if (m != 0) {
        const u32 nch = (st->ncols + cpc - 1) / cpc;
        u64 s0 = 0, s1 = 0;
        for (u32 c = 0; c < nch; ++c) {
          const u64 b0 = cnt0[(size_t)c * Ls + w], b1 = cnt1[(size_t)c * Ls + w];
          const u64 carry = s0 & b0;
          s0 ^= b0;
          s1 ^= b1 ^ carry;
        }
        if (s0 & m) atomicOr(&st->flags, 1u);
        r ^= m & (s1 ^ (rp ? ~0ULL : 0ULL));
      }
      if (w == wd) r = (r & ~bit) | (rp ? bit : 0ULL);
      if (w == ws) r = (r & ~bit) | (st->coin ? bit : 0ULL);
      R[w] = r;
    }
  }
  if (tid < n) {
    const u32 j = tid;
    const u64 xb = (pivx[j >> 6] >> (j & 63u)) & 1ULL, zb = (pivz[j >> 6] >> (j & 63u)) & 1ULL;
    u64 *x = X + (size_t)j * Ls;
    u64 *z = Z + (size_t)j * Ls;
    x[wd] = (x[wd] & ~bit) | (xb ? bit : 0ULL);
    z[wd] = (z[wd] & ~bit) | (zb ? bit : 0ULL);
    x[ws] &= ~bit;
    z[ws] = (z[ws] & ~bit) | ((j == q) ? bit : 0ULL);
  }
}

// ---------------------------------------------------------------------------
// a6: deterministic outcome. A = {i : x(D_i)_q = 1} (the destabilizer half of
// the mask). The product of S_i over i in A, taken in ascending i, is
// +-Z_q. Per column j, the running product before row i has x/z bits equal
// to the exclusive prefix XOR over A of the stabilizer bits of column j; so
// the phase exponent adds g(P_ij, prefix) for each i in A. A workgroup walks
// each of its columns in rounds of blockDim*WPT words; the prefix across
// words is a wave ballot scan plus a cross-wave LDS scan plus the carry of
// earlier rounds. The column's total XOR must be 0 for x and [j == q] for z.
__device__ __forceinline__ u64 prefix_xor_incl(u64 v) {
  v ^= v << 1;
  v ^= v << 2;
  v ^= v << 4;
  v ^= v << 8;
  v ^= v << 16;
  v ^= v << 32;
  return v;
}

template <int WPT>
__global__ __launch_bounds__(1024) void k_detphase(const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                                    const u64 *__restrict__ mask, MeasState *__restrict__ st, u32 Ls,
                                                    u32 K, u32 n, u32 q, u32 cpw) {
  if (st->p >= 0) return;
  __shared__ u32 s_px[16], s_pz[16];
  __shared__ int s_acc[16];
  const u32 tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
  int acc = 0;
  u32 bad = 0;
  const u32 j0 = blockIdx.x * cpw, j1 = min(j0 + cpw, n);
  for (u32 j = j0; j < j1; ++j) {
    const u64 *xc = X + (size_t)j * Ls + K;
    const u64 *zc = Z + (size_t)j * Ls + K;
    u32 carry_x = 0, carry_z = 0;
    for (u32 base = 0; base < K; base += blockDim.x * WPT) {
      const u32 w0 = base + tid * WPT;
      u64 sx[WPT], sz[WPT];
      u32 tpx = 0, tpz = 0;
#pragma unroll
      for (int k = 0; k < WPT; ++k) {
        const u32 w = w0 + k;
        const u64 a = (w < K) ? mask[w] : 0ULL;
        sx[k] = a ? (xc[w] & a) : 0ULL;
        sz[k] = a ? (zc[w] & a) : 0ULL;
        tpx ^= (u32)__popcll(sx[k]) & 1u;
        tpz ^= (u32)__popcll(sz[k]) & 1u;
      }
      const u64 bx = __ballot(tpx), bz = __ballot(tpz);
      if (lane == 0) {
        s_px[wave] = (u32)__popcll(bx) & 1u;
        s_pz[wave] = (u32)__popcll(bz) & 1u;
      }
      __syncthreads();
      u32 cx = carry_x ^ ((u32)__popcll(bx & lanemask_lt()) & 1u);
      u32 cz = carry_z ^ ((u32)__popcll(bz & lanemask_lt()) & 1u);
      for (u32 v = 0; v < nwaves; ++v) {
        if (v < wave) { cx ^= s_px[v]; cz ^= s_pz[v]; }
        carry_x ^= s_px[v];
        carry_z ^= s_pz[v];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < WPT; ++k) {
        const u64 ex = (prefix_xor_incl(sx[k]) << 1) ^ (cx ? ~0ULL : 0ULL);
        const u64 ez = (prefix_xor_incl(sz[k]) << 1) ^ (cz ? ~0ULL : 0ULL);
        const u64 x1 = sx[k], z1 = sz[k];
        const u64 p_x = x1 & ~z1, p_y = x1 & z1, p_z = ~x1 & z1;
        const u64 plus = (p_x & ex & ez) | (p_y & ~ex & ez) | (p_z & ex & ~ez);
        const u64 minus = (p_x & ~ex & ez) | (p_y & ex & ~ez) | (p_z & ex & ez);
        acc += __popcll(plus) - __popcll(minus);
        cx ^= (u32)__popcll(sx[k]) & 1u;
        cz ^= (u32)__popcll(sz[k]) & 1u;
      }
    }
    if (carry_x != 0u || carry_z != (u32)(j == q)) bad = 1;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) s_acc[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (u32 v = 0; v < nwaves; ++v) tot += s_acc[v];
    atomicAdd(&st->det_acc, (u32)tot);
    if (bad) atomicOr(&st->flags, 2u);
  }
}

// Outcome = parity of the signs of S_i over A, xor bit 1 of the phase sum
// (which must be even).
__global__ __launch_bounds__(256) void k_detfinal(const u64 *__restrict__ R, const u64 *__restrict__ mask,
                                                  MeasState *__restrict__ st, MeasStats *__restrict__ stats, u32 K,
                                                  u32 n, uint8_t *__restrict__ out_bits) {
  if (st->p >= 0) return;
  __shared__ u32 s_par[4];
  const u32 tid = threadIdx.x;
  u32 par = 0;
  for (u32 w = tid; w < K; w += blockDim.x) par ^= (u32)__popcll(R[K + w] & mask[w]) & 1u;
  const u64 b = __ballot(par);
  if ((tid & 63u) == 0) s_par[tid >> 6] = (u32)__popcll(b) & 1u;
  __syncthreads();
  if (tid == 0) {
    u32 tot = 0;
    for (u32 v = 0; v < (blockDim.x >> 6); ++v) tot ^= s_par[v];
    const u32 e = st->det_acc & 3u;
    if (e & 1u) atomicOr(&st->flags, 1u);
    out_bits[0] = (uint8_t)(tot ^ (e >> 1));
    // Algorithmic bytes: x and z of every column at each word holding a row of A.
    stats->n_det += 1;
    stats->det_bytes += (u64)st->awords * 8ULL * 2ULL * n;
  }
}

// ---------------------------------------------------------------------------
// Canonical row-major export/import (checks and checkpoints; not a hot path).
__global__ void k_export_rows(const u64 *__restrict__ X, const u64 *__restrict__ Z, const u64 *__restrict__ R,
                              u32 Ls, u32 K, u32 n, const u32 *__restrict__ rows, u32 nrows, u32 W,
                              u64 *__restrict__ ox, u64 *__restrict__ oz, uint8_t *__restrict__ orr) {
  const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
  for (u32 k = blockIdx.y; k < nrows; k += gridDim.y) {
    const u32 g = rows[k];
    const u32 wr = (g < n) ? (g >> 6) : (K + ((g - n) >> 6));
    const u32 br = ((g < n) ? g : (g - n)) & 63u;
    u32 xb = 0, zb = 0;
    if (j < n) {
      xb = (u32)(X[(size_t)j * Ls + wr] >> br) & 1u;
      zb = (u32)(Z[(size_t)j * Ls + wr] >> br) & 1u;
    }
    const u64 bx = __ballot(xb), bz = __ballot(zb);
    if ((threadIdx.x & 63u) == 0 && (j >> 6) < W) {
      ox[(size_t)k * W + (j >> 6)] = bx;
      oz[(size_t)k * W + (j >> 6)] = bz;
    }
    if (j == 0) orr[k] = (uint8_t)((R[wr] >> br) & 1ULL);
  }
}

// Column word (j, w) gathers bit j of the 64 rows that word w packs.
__global__ void k_import(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ R, u32 Ls, u32 K, u32 L, u32 n,
                         const u64 *__restrict__ ix, const u64 *__restrict__ iz, const uint8_t *__restrict__ ir,
                         u32 W, u32 wblocks) {
  const u32 j = blockIdx.x / wblocks;
  const u32 w = (blockIdx.x % wblocks) * blockDim.x + threadIdx.x;
  if (w >= L) return;
  const u32 half = (w < K) ? 0u : n;
  const u32 r0 = ((w < K) ? w : (w - K)) * 64u;
  u64 vx = 0, vz = 0, vr = 0;
  for (u32 b = 0; b < 64u && r0 + b < n; ++b) {
    const size_t g = (size_t)half + r0 + b;
    vx |= ((ix[g * W + (j >> 6)] >> (j & 63u)) & 1ULL) << b;
    vz |= ((iz[g * W + (j >> 6)] >> (j & 63u)) & 1ULL) << b;
    if (j == 0) vr |= (u64)(ir[g] & 1u) << b;
  }
  X[(size_t)j * Ls + w] = vx;
  Z[(size_t)j * Ls + w] = vz;
  if (j == 0) R[w] = vr;
}

// ---------------------------------------------------------------------------
// Launchers.
static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

hipError_t launch_fill_zero(u64 *p, size_t words, hipStream_t s) {
  if (words == 0) return hipSuccess;
  const u32 blocks = (u32)std::min<u64>(cdiv(words, 256), 65536);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, p, words);
  return hipGetLastError();
}

hipError_t launch_init_diag(const TabDev &t, hipStream_t s) {
  hipLaunchKernelGGL(k_init_diag, dim3(cdiv(t.n, 256)), dim3(256), 0, s, t.X, t.Z, t.n, t.K, t.Ls);
  return hipGetLastError();
}

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

hipError_t launch_pivot(const TabDev &t, u32 q, MeasState *st, u64 *mask, u64 seed, u64 shot, u64 m,
                        uint8_t *out_bits, uint8_t *out_rand, hipStream_t s) {
  hipLaunchKernelGGL(k_pivot, dim3(1), dim3(1024), 0, s, t.X, t.Ls, t.K, t.L, q, st, mask, seed, shot, m, out_bits,
                     out_rand);
  return hipGetLastError();
}

hipError_t launch_gather(const TabDev &t, MeasState *st, u64 *pivx, u64 *pivz, u32 *cols, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(cdiv(t.n, 256)), dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st, pivx, pivz,
                     cols);
  return hipGetLastError();
}

hipError_t launch_rowsum(const TabDev &t, const u64 *mask, const u32 *cols, const MeasState *st, u64 *cnt0,
                         u64 *cnt1, u32 block, u32 wpt, u32 cpc, u32 max_chunks, hipStream_t s) {
  const u32 tiles = cdiv(t.L, (u64)block * wpt);
  dim3 grid(tiles, max_chunks);
  if (wpt == 2)
    hipLaunchKernelGGL((k_rowsum<2, 4>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1, t.Ls, t.L,
                       cpc);
  else
    hipLaunchKernelGGL((k_rowsum<1, 4>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1, t.Ls, t.L,
                       cpc);
  return hipGetLastError();
}

hipError_t launch_finalize(const TabDev &t, u32 q, const u64 *mask, const u64 *pivx, const u64 *pivz,
                           const u64 *cnt0, const u64 *cnt1, MeasState *st, MeasStats *stats, u32 cpc,
                           hipStream_t s) {
  const u32 threads = std::max(t.L, t.n);
  hipLaunchKernelGGL(k_finalize, dim3(cdiv(threads, 256)), dim3(256), 0, s, t.X, t.Z, t.R, mask, pivx, pivz, cnt0,
                     cnt1, st, stats, t.Ls, t.L, t.K, t.n, q, cpc);
  return hipGetLastError();
}

hipError_t launch_detphase(const TabDev &t, u32 q, const u64 *mask, MeasState *st, u32 block, u32 cols_per_wg,
                           hipStream_t s) {
  hipLaunchKernelGGL((k_detphase<2>), dim3(cdiv(t.n, cols_per_wg)), dim3(block), 0, s, t.X, t.Z, mask, st, t.Ls,
                     t.K, t.n, q, cols_per_wg);
  return hipGetLastError();
}

hipError_t launch_detfinal(const TabDev &t, const u64 *mask, MeasState *st, MeasStats *stats, uint8_t *out_bits,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_detfinal, dim3(1), dim3(256), 0, s, t.R, mask, st, stats, t.K, t.n, out_bits);
  return hipGetLastError();
}

hipError_t launch_export_rows(const TabDev &t, const u32 *rows, u32 nrows, u32 W, u64 *ox, u64 *oz, uint8_t *orr,
                              hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  const u32 cols_rounded = W * 64u;
  dim3 grid(cdiv(cols_rounded, 256), std::min<u32>(nrows, 65535u));
  hipLaunchKernelGGL(k_export_rows, grid, dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, rows, nrows, W, ox, oz,
                     orr);
  return hipGetLastError();
}

hipError_t launch_import(const TabDev &t, const u64 *ix, const u64 *iz, const uint8_t *ir, u32 W, hipStream_t s) {
  const u32 wblocks = cdiv(t.L, 256);
  hipLaunchKernelGGL(k_import, dim3(wblocks * t.n), dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.L, t.n, ix, iz, ir,
                     W, wblocks);
  return hipGetLastError();
}

}  // namespace sq
