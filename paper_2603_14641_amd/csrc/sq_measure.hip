// Z measurement (CHP), four launches per measured qubit:
//   k_pivot  (a3)  pivot search, rowsum mask snapshot, coin;
//   k_gather (a4)  pivot row S_p packed and its non-identity columns compacted;
//   k_rowsum (a5)  every anticommuting row times S_p with the exact phase;
//   k_post   (a5/a6) random case: signs from the phase counters, D_p <- S_p,
//            S_p <- +-Z_q; deterministic case: the ordered product of the
//            stabilizers that A selects, whose sign is the outcome.
// The same kernels serve the symbolic-sign sweep of the sampler (SYM), in
// which stabilizer signs are affine forms over the coins (see sq_sample.hip).
#include "sq_device.h"

namespace sq {

constexpr u32 SIGN_COLS_PER_BLOCK = 32;  // coin columns per sign-XOR block of k_rowsum

// ---------------------------------------------------------------------------
// a3: pivot search for measuring qubit q = list[i] alone, i the cursor's
// position: with kb == 1 every slot measures its list entry this way; with
// blocks only the deterministic measurement that ended the slot's block does
// (the cursor's `single` flag), and any other slot measures nothing
// (MeasState::p = P_NONE, which the slot's later kernels skip). p = the
// smallest stabilizer index with x(S_p)_q = 1 (first set bit of the
// stabilizer half of X column q), or -1. Also snapshots column q into `mask`
// (the rows the rowsum pass must touch), with the bits of D_p and S_p
// cleared, because the pass rewrites column q in place. With no pivot (the
// deterministic case) it also lists the nonzero destabilizer-half words of
// column q in ascending order: alist[e] = word index, amask[e] = its bits
// (the rows of A), e < awords. One workgroup; thread 0 also draws the coin
// and advances the cursor.
__global__ __launch_bounds__(1024) void k_pivot(const u64 *__restrict__ X, u32 Ls, u32 K, u32 L,
                                                Cursor *__restrict__ cur, MeasState *__restrict__ st,
                                                u64 *__restrict__ mask, u32 *__restrict__ alist,
                                                u64 *__restrict__ amask) {
  __shared__ u32 s_min, s_act, s_q, s_i;
  const u32 tid = threadIdx.x;
  if (tid == 0) {
    s_min = 0xFFFFFFFFu;
    const u32 i = cur->i;
    const u32 act = cur->kb <= 1u ? (i < cur->end ? 1u : 0u) : cur->single;
    s_act = act;
    s_i = i;
    s_q = act ? cur->qubits[i] : 0u;
  }
  __syncthreads();
  if (!s_act) {
    if (tid == 0) st->p = P_NONE;
    return;
  }
  const u32 q = s_q, i = s_i;
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
  // (thread 0 may set p to P_NONE below; the snapshot uses the pivot found)
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
  if (p < 0) {  // uniform: p comes from s_min
    // ordered compaction, one round of blockDim words at a time: wave ballot
    // rank plus the counts of the lower waves and of earlier rounds
    __shared__ u32 s_wc[16];
    const u32 wave = tid >> 6, nwaves = blockDim.x >> 6;
    u32 base = 0;
    for (u32 r0 = 0; r0 < K; r0 += blockDim.x) {
      const u32 w = r0 + tid;
      const u64 v = (w < K) ? col[w] : 0ULL;
      const u64 b = __ballot(v != 0);
      if ((tid & 63u) == 0) s_wc[wave] = (u32)__popcll(b);
      __syncthreads();
      u32 e = base + (u32)__popcll(b & lanemask_lt()), tot = 0;
      for (u32 u = 0; u < nwaves; ++u) {
        if (u < wave) e += s_wc[u];
        tot += s_wc[u];
      }
      if (v != 0) {
        alist[e] = w;
        amask[e] = v;
      }
      base += tot;
      __syncthreads();  // s_wc is rewritten in the next round
    }
  }
  if (tid == 0) {
    const u32 c = coin_bit(cur->seed, cur->shot, cur->meas_base + i);
    const bool blocked = cur->kb > 1u;
    if (blocked && p >= 0) {
      // the blocked pivot step found no pivot for this measurement: the two
      // searches disagree, which is a bug; flag it and measure nothing
      atomicOr(&st->flags, 4u);
      p = P_NONE;
    }
    st->p = p;
    st->q = q;
    st->i = i;
    st->ncols = 0;
    st->nsv = 0;
    st->nx = 0;
    st->nz = 0;
    st->mwords = s_mw;
    st->awords = s_aw;
    st->det_acc = 0;
    st->det_done = 0;
    st->coin = c;
    if (p != P_NONE && cur->out_rand) cur->out_rand[i] = (uint8_t)(p >= 0);
    if (p >= 0 && cur->out_bits) cur->out_bits[i] = (uint8_t)c;
    cur->i = i + 1;
    cur->single = 0;
  }
}

// a4: gather the pivot row S_p across all columns (one 8-byte read per column),
// pack it with wave ballots into pivx/pivz (bit j of word j/64), and compact
// the columns where S_p is not the identity into `cols`
// (entry = j | x_pj << 31 | z_pj << 30; order across waves is arbitrary).
// r_p (st->rp) is S_p's sign, or in the sampler S_p's constant sign term; the
// sampler's extra blocks compact the coins v < i in whose sign column S_p has
// a 1 into svlist.
template <bool SYM>
__global__ void k_gather(const u64 *__restrict__ X, const u64 *__restrict__ Z, const u64 *__restrict__ R, u32 Ls,
                         u32 K, u32 n, MeasState *__restrict__ st, u64 *__restrict__ pivx, u64 *__restrict__ pivz,
                         u32 *__restrict__ cols, SymCtx sym) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 ws = K + ((u32)p >> 6), sh = (u32)p & 63u;
  const u32 lane = threadIdx.x & 63u;
  const u32 colblocks = (n + blockDim.x - 1) / blockDim.x;
  if (SYM && blockIdx.x >= colblocks) {
    const u32 v = (blockIdx.x - colblocks) * blockDim.x + threadIdx.x;
    const u32 b = (v < st->i) ? (u32)(sym.sg[(size_t)v * sym.Ks + ((u32)p >> 6)] >> sh) & 1u : 0u;
    const u64 bb = __ballot(b);
    u32 base = 0;
    if (lane == 0 && bb) base = atomicAdd(&st->nsv, (u32)__popcll(bb));
    base = (u32)__shfl((int)base, 0);
    if (b) sym.svlist[base + (u32)__popcll(bb & lanemask_lt())] = v;
    return;
  }
  const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
  u32 xb = 0, zb = 0;
  if (j < n) {
    xb = (u32)(X[(size_t)j * Ls + ws] >> sh) & 1u;
    zb = (u32)(Z[(size_t)j * Ls + ws] >> sh) & 1u;
  }
  const u64 bx = __ballot(xb), bz = __ballot(zb);
  const u64 nz = bx | bz;
  u32 base = 0;
  if (lane == 0) {
    if (j < n) { pivx[j >> 6] = bx; pivz[j >> 6] = bz; }
    if (nz) base = atomicAdd(&st->ncols, (u32)__popcll(nz));
    if (bx) atomicAdd(&st->nx, (u32)__popcll(bx));
    if (bz) atomicAdd(&st->nz, (u32)__popcll(bz));
  }
  base = (u32)__shfl((int)base, 0);
  if (xb | zb) cols[base + (u32)__popcll(nz & lanemask_lt())] = j | (xb << 31) | (zb << 30);
  if (j == 0) {
    const u64 *sw = SYM ? (sym.sg + (size_t)sym.count * sym.Ks + ((u32)p >> 6)) : (R + ws);
    st->rp = (u32)(*sw >> sh) & 1u;
  }
}

// a5: random-case rowsum pass. For every masked row h (x_hq = 1, h not D_p or
// S_p): row_h <- S_p * row_h. Per non-identity pivot column j with Pauli P1
// = (x_pj, z_pj): x_h ^= x_pj, z_h ^= z_pj, and the phase exponent
// g(P1, P_hj) in {-1, 0, +1} is added to a bit-sliced 2-bit counter per row
// (a0 = bit 0, a1 = bit 1). g is +1 for (X,Y), (Y,Z), (Z,X) and -1 for
// (X,Z), (Y,X), (Z,Y). Counters of each column chunk go to cnt0/cnt1.
// Sampling (SYM): rows blockIdx.y >= rchunks of the grid instead XOR the
// rowsum mask of the stabilizer half into every coin column in which S_p has
// a 1 (the masked stabilizers take S_p's sign vector; its constant term is
// folded in by k_post like r_p).
template <int WPT, int B, bool SYM>
__global__ __launch_bounds__(1024) void k_rowsum(u64 *__restrict__ X, u64 *__restrict__ Z,
                                                  const u64 *__restrict__ mask, const u32 *__restrict__ cols,
                                                  const MeasState *__restrict__ st, u64 *__restrict__ cnt0,
                                                  u64 *__restrict__ cnt1, u32 Ls, u32 L, u32 cpc, u32 rchunks,
                                                  SymCtx sym) {
  if (st->p < 0) return;
  if (SYM && blockIdx.y >= rchunks) {
    const u32 nsv = st->nsv;
    const u32 v0 = (blockIdx.y - rchunks) * SIGN_COLS_PER_BLOCK;
    if (v0 >= nsv) return;
    const u32 v1 = min(v0 + SIGN_COLS_PER_BLOCK, nsv);
    const u32 K = L / 2;
    const u32 wb = (blockIdx.x * blockDim.x + threadIdx.x) * WPT;
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
      const u32 w = wb + k;
      if (w >= K) break;
      const u64 m = mask[K + w];
      if (m == 0) continue;
      for (u32 v = v0; v < v1; ++v) sym.sg[(size_t)sym.svlist[v] * sym.Ks + w] ^= m;
    }
    return;
  }
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
      ldw_nt<WPT>(X + o, x[b]);
      ldw_nt<WPT>(Z + o, z[b]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      step(e[b], x[b], z[b]);
      const size_t o = (size_t)(e[b] & 0x3FFFFFFFu) * Ls + w;
      if (e[b] >> 31) {
        u64 v[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) v[k] = x[b][k] ^ m[k];
        stw_nt<WPT>(X + o, v);
      }
      if ((e[b] >> 30) & 1u) {
        u64 v[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) v[k] = z[b][k] ^ m[k];
        stw_nt<WPT>(Z + o, v);
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

// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 prefix_xor_incl(u64 v) {
  v ^= v << 1;
  v ^= v << 2;
  v ^= v << 4;
  v ^= v << 8;
  v ^= v << 16;
  v ^= v << 32;
  return v;
}

// The deterministic product's column walk (k_post): list entries per lane
// per round when A's words take more than one wave-wide step, and columns
// whose loads are issued together when they fit in one.
constexpr u32 DET_U = 4;
constexpr u32 DET_CB = 4;

// One word of a deterministic product in a column: x1/z1 are the column's
// stabilizer bits at 64 rows of A (zero outside A), one word per lane in
// ascending row order across the wave; cx/cz the XOR of the column's bits over
// the rows of A before this wave-wide word group. The running product before
// row i has x/z equal to that carry plus the exclusive prefix XOR inside the
// word group, and S_i's phase contribution against it is +1, -1 or 0 (the
// g function of the rowsum). Call with the whole wave.
__device__ __forceinline__ void det_word(u64 x1, u64 z1, u32 &cx, u32 &cz, int &acc) {
  const u64 bx = __ballot(__popcll(x1) & 1), bz = __ballot(__popcll(z1) & 1);
  const u64 lt = lanemask_lt();
  const u32 px = cx ^ ((u32)__popcll(bx & lt) & 1u), pz = cz ^ ((u32)__popcll(bz & lt) & 1u);
  const u64 ex = (prefix_xor_incl(x1) << 1) ^ (px ? ~0ULL : 0ULL);
  const u64 ez = (prefix_xor_incl(z1) << 1) ^ (pz ? ~0ULL : 0ULL);
  const u64 p_x = x1 & ~z1, p_y = x1 & z1, p_z = ~x1 & z1;
  const u64 plus = (p_x & ex & ez) | (p_y & ~ex & ez) | (p_z & ex & ~ez);
  const u64 minus = (p_x & ~ex & ez) | (p_y & ex & ~ez) | (p_z & ex & ez);
  acc += __popcll(plus) - __popcll(minus);
  cx ^= (u32)__popcll(bx) & 1u;
  cz ^= (u32)__popcll(bz) & 1u;
}

// k_post. Random case (p >= 0), by global thread index t:
//   * t < L (plain) or t < K (sampler): for a masked row word, add the chunk
//     counters mod 4; the exponent 2 r_h + 2 r_p + sum g must be even and
//     r_h <- r_h ^ r_p ^ bit1(sum g). D_p's sign <- r_p, S_p's <- coin (plain);
//     the sampler updates the constant column and clears S_p's constant bit;
//   * t < n: column t's bits of D_p <- S_p's, S_p <- Z_q;
//   * sampler, t < nsv: clear S_p's bit in the listed coin columns; t = 0 sets
//     coin column i (S_p's sign is now coin i).
// Deterministic case (p < 0): A = {i : x(D_i)_q = 1} (destabilizer half of
// the mask). The product of S_i over A in ascending i is +-Z_q. Per column j
// the running product before row i has x/z bits equal to the exclusive prefix
// XOR over A of column j's stabilizer bits, so the phase exponent adds
// g(P_ij, prefix) for each i in A. Block b takes columns [b*cpw, (b+1)*cpw),
// its waves one column at a time each; a wave walks only the words of A that
// k_pivot listed (alist/amask), 64 per wave-wide step (det_word), so a column
// costs the bytes of A's words, not of all K. The column's total XOR
// must be 0 for x and [j == q] for z. Blocks add their sums into the ticket
// word det_done; the last block to finish (no waiting) forms the outcome:
// parity of S_i's signs over A xor bit 1 of the sum (which must be even). The
// sampler's blocks also compute the coin coefficients of the outcome's affine form
// (parity of sign column v over A, v < i), and the last block its constant.
template <bool SYM>
__global__ __launch_bounds__(256) void k_post(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ R,
                                              const u64 *__restrict__ mask, const u64 *__restrict__ pivx,
                                              const u64 *__restrict__ pivz, const u64 *__restrict__ cnt0,
                                              const u64 *__restrict__ cnt1, const u32 *__restrict__ alist,
                                              MeasState *__restrict__ st, MeasStats *__restrict__ stats,
                                              const Cursor *__restrict__ cur, u32 Ls, u32 L, u32 K, u32 n, u32 cpc,
                                              u32 cpw, SymCtx sym) {
  const int32_t p = st->p;
  if (p == P_NONE) return;  // the slot measures nothing alone
  const u32 q = st->q, li = st->i;  // the qubit and its list position
  const u32 tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const u32 t = blockIdx.x * blockDim.x + tid;
  if (p >= 0) {
    const u32 wd = (u32)p >> 6, ws = K + wd;
    const u64 bit = 1ULL << ((u32)p & 63u);
    const u32 rp = st->rp;
    if (t == 0 && !SYM) {
      // Algorithmic bytes of this rowsum: every touched row word reads x and z
      // of each non-identity pivot column and writes x (if x_pj) and z (if z_pj).
      stats->n_random += 1;
      stats->rowsum_bytes += (u64)st->mwords * 8ULL * (2ULL * st->ncols + st->nx + st->nz);
    }
    // Sign words: one wave per row word; lanes sum the chunks' 2-bit
    // counters over a stride of 64 chunks, then a butterfly adds the lanes'
    // counters (bit-sliced, mod 4).
    const u32 nsign = SYM ? K : L;
    const u32 gw = blockIdx.x * nwaves + wave;
    if (gw < nsign) {
      const u32 w = SYM ? K + gw : gw;  // row word
      const u64 m = mask[w];
      const bool own = SYM ? (w == ws) : (w == wd || w == ws);
      if (m != 0 || own) {  // uniform over the wave
        u64 s0 = 0, s1 = 0;
        if (m != 0) {
          const u32 nch = (st->ncols + cpc - 1) / cpc;
          for (u32 c = lane; c < nch; c += 64u) {
            const u64 b0 = cnt0[(size_t)c * Ls + w], b1 = cnt1[(size_t)c * Ls + w];
            const u64 carry = s0 & b0;
            s0 ^= b0;
            s1 ^= b1 ^ carry;
          }
          for (int off = 32; off > 0; off >>= 1) {
            const u64 o0 = shfl_xor_u64(s0, off), o1 = shfl_xor_u64(s1, off);
            const u64 carry = s0 & o0;
            s0 ^= o0;
            s1 ^= o1 ^ carry;
          }
        }
        if (lane == 0) {
          u64 r = SYM ? sym.sg[(size_t)sym.count * sym.Ks + gw] : R[w];
          if (m != 0) {
            if (s0 & m) atomicOr(&st->flags, 1u);
            r ^= m & (s1 ^ (rp ? ~0ULL : 0ULL));
          }
          if (SYM) {
            if (w == ws) r &= ~bit;
            sym.sg[(size_t)sym.count * sym.Ks + gw] = r;
          } else {
            if (w == wd) r = (r & ~bit) | (rp ? bit : 0ULL);
            if (w == ws) r = (r & ~bit) | (st->coin ? bit : 0ULL);
            R[w] = r;
          }
        }
      }
    }
    if (t < n) {
      const u32 j = t;
      const u64 xb = (pivx[j >> 6] >> (j & 63u)) & 1ULL, zb = (pivz[j >> 6] >> (j & 63u)) & 1ULL;
      u64 *x = X + (size_t)j * Ls;
      u64 *z = Z + (size_t)j * Ls;
      x[wd] = (x[wd] & ~bit) | (xb ? bit : 0ULL);
      z[wd] = (z[wd] & ~bit) | (zb ? bit : 0ULL);
      x[ws] &= ~bit;
      z[ws] = (z[ws] & ~bit) | ((j == q) ? bit : 0ULL);
    }
    if (SYM) {
      if (t < st->nsv) sym.sg[(size_t)sym.svlist[t] * sym.Ks + wd] &= ~bit;
      if (t == 0) {
        sym.sg[(size_t)li * sym.Ks + wd] |= bit;
        sym.kind[li] = 1;
      }
    }
    return;
  }

  // ---- deterministic case
  __shared__ u32 s_px[4], s_last, s_e;
  __shared__ int s_acc[4];
  const u32 aw = st->awords;
  const u64 *amask = pivx;  // the compacted rows of A (k_pivot; pivx is free here)
  int acc = 0;
  u32 bad = 0;
  const u32 j0 = blockIdx.x * cpw, j1 = min(j0 + cpw, n);
  if (aw <= 64u) {
    // A within one round: the list is loop-invariant, and DET_CB columns'
    // loads are issued before any of their scans
    const bool on = lane < aw;
    const u32 w = on ? alist[lane] : 0u;
    const u64 a = on ? amask[lane] : 0ULL;
    for (u32 j = j0 + wave; j < j1; j += DET_CB * nwaves) {
      u64 sx[DET_CB], sz[DET_CB];
#pragma unroll
      for (u32 k = 0; k < DET_CB; ++k) {
        const u32 jj = j + k * nwaves;
        const bool ok = on && jj < j1;
        sx[k] = ok ? (X[(size_t)jj * Ls + K + w] & a) : 0ULL;
        sz[k] = ok ? (Z[(size_t)jj * Ls + K + w] & a) : 0ULL;
      }
#pragma unroll
      for (u32 k = 0; k < DET_CB; ++k) {
        const u32 jj = j + k * nwaves;
        if (jj < j1) {  // uniform over the wave
          u32 cx = 0, cz = 0;
          det_word(sx[k], sz[k], cx, cz, acc);
          if (cx != 0u || cz != (u32)(jj == q)) bad = 1;
        }
      }
    }
  } else {
    // rounds of DET_U list entries per lane (entry base + k*64 + lane), the
    // loads of a round issued before its scans
    for (u32 j = j0 + wave; j < j1; j += nwaves) {
      const u64 *xc = X + (size_t)j * Ls + K;
      const u64 *zc = Z + (size_t)j * Ls + K;
      u32 cx = 0, cz = 0;
      for (u32 base = 0; base < aw; base += 64u * DET_U) {
        u64 sx[DET_U], sz[DET_U];
#pragma unroll
        for (u32 k = 0; k < DET_U; ++k) {
          const u32 e = base + k * 64u + lane;
          sx[k] = 0;
          sz[k] = 0;
          if (e < aw) {
            const u32 w = alist[e];
            const u64 a = amask[e];
            sx[k] = xc[w] & a;
            sz[k] = zc[w] & a;
          }
        }
#pragma unroll
        for (u32 k = 0; k < DET_U; ++k) det_word(sx[k], sz[k], cx, cz, acc);
      }
      if (cx != 0u || cz != (u32)(j == q)) bad = 1;
    }
  }
  if (SYM) {
    // Coin coefficients of the outcome's affine form: bit v of F_i is the
    // parity of sign column v over the rows in A (v < i). Block b builds
    // word b (columns 64b .. 64b+63); each wave takes 64 / nwaves columns and
    // reads a column's words lane by lane (coalesced).
    // (k_post runs with 256 threads: 4 waves of 16 columns; a lane loads its
    // word of all 16 columns before using any, so a wave waits about K / 64
    // memory round trips, not 16 times that)
    constexpr u32 PER = 16;
    __shared__ u64 s_fw;
    if (tid == 0) s_fw = 0;
    __syncthreads();
    const u32 vbase = blockIdx.x * 64u;
    const u32 v0 = vbase + wave * PER;
    if (v0 < li) {
      u32 par[PER];
#pragma unroll
      for (u32 k = 0; k < PER; ++k) par[k] = 0;
      for (u32 e = lane; e < aw; e += 64u) {
        const u32 w = alist[e];
        const u64 m = amask[e];
        u64 c[PER];
#pragma unroll
        for (u32 k = 0; k < PER; ++k) c[k] = (v0 + k < li) ? sym.sg[(size_t)(v0 + k) * sym.Ks + w] : 0ULL;
#pragma unroll
        for (u32 k = 0; k < PER; ++k) par[k] ^= (u32)__popcll(c[k] & m) & 1u;
      }
      u64 bits = 0;
#pragma unroll
      for (u32 k = 0; k < PER; ++k) bits |= (u64)((u32)__popcll(__ballot(par[k])) & 1u) << k;
      if (lane == 0 && bits) atomicOr(&s_fw, bits << (v0 & 63u));
    }
    __syncthreads();
    if (tid == 0 && vbase <= li) sym.fm[(size_t)li * sym.CW + blockIdx.x] = s_fw;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) s_acc[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (u32 v = 0; v < nwaves; ++v) tot += s_acc[v];
    if (bad) atomicOr(&st->flags, 2u);
    // One atomic carries both the ticket (bits 0..23: blocks done) and the
    // phase sum (bits 24..31, mod 256: only its value mod 4 is used), so the
    // last block has the whole sum without a device-scope fence per block.
    const u32 old = atomicAdd(&st->det_done, 1u + ((u32)tot << 24));
    s_last = ((old & 0xFFFFFFu) == gridDim.x - 1) ? 1u : 0u;
    s_e = ((old >> 24) + (u32)tot) & 3u;
  }
  __syncthreads();
  if (!s_last) return;
  // last block: sign parity over A, then the outcome (or the constant of its affine form)
  u32 par = 0;
  const u64 *sgn = SYM ? (sym.sg + (size_t)sym.count * sym.Ks) : (R + K);
  for (u32 e = tid; e < aw; e += blockDim.x) par ^= (u32)__popcll(sgn[alist[e]] & amask[e]) & 1u;
  const u64 b = __ballot(par);
  if (lane == 0) s_px[wave] = (u32)__popcll(b) & 1u;
  __syncthreads();
  if (tid == 0) {
    u32 tot = 0;
    for (u32 v = 0; v < nwaves; ++v) tot ^= s_px[v];
    const u32 e = s_e;
    if (e & 1u) atomicOr(&st->flags, 1u);
    const uint8_t outcome = (uint8_t)(tot ^ (e >> 1));
    if (SYM) {
      sym.fc[li] = outcome;
      sym.kind[li] = 0;
    } else {
      if (cur->out_bits) cur->out_bits[li] = outcome;
      // Algorithmic bytes: x and z of every column at each word holding a row of A.
      stats->n_det += 1;
      stats->det_bytes += (u64)st->awords * 8ULL * 2ULL * n;
    }
  }
}

// Launchers.
__global__ void k_cursor_init(Cursor *c, u32 end, u32 kb, u64 seed, u64 shot, u64 meas_base, const u32 *qubits,
                              uint8_t *out_bits, uint8_t *out_rand) {
  if (threadIdx.x == 0) {
    c->i = 0;
    c->end = end;
    c->kb = kb;
    c->single = 0;
    c->seed = seed;
    c->shot = shot;
    c->meas_base = meas_base;
    c->qubits = qubits;
    c->out_bits = out_bits;
    c->out_rand = out_rand;
  }
}

hipError_t launch_cursor_init(Cursor *c, u32 end, u32 kb, u64 seed, u64 shot, u64 meas_base, const u32 *qubits,
                              uint8_t *out_bits, uint8_t *out_rand, hipStream_t s) {
  hipLaunchKernelGGL(k_cursor_init, dim3(1), dim3(64), 0, s, c, end, kb, seed, shot, meas_base, qubits, out_bits,
                     out_rand);
  return hipGetLastError();
}

hipError_t launch_pivot(const TabDev &t, Cursor *cur, MeasState *st, u64 *mask, u32 *alist, u64 *amask,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_pivot, dim3(1), dim3(1024), 0, s, t.X, t.Ls, t.K, t.L, cur, st, mask, alist, amask);
  return hipGetLastError();
}

hipError_t launch_gather(const TabDev &t, MeasState *st, u64 *pivx, u64 *pivz, u32 *cols, const SymCtx *sym,
                         hipStream_t s) {
  const u32 colblocks = cdiv(t.n, 256);
  if (sym) {
    const u32 vblocks = cdiv(sym->count, 256);  // coin columns before the measurement's position
    hipLaunchKernelGGL(k_gather<true>, dim3(colblocks + vblocks), dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st,
                       pivx, pivz, cols, *sym);
  } else {
    hipLaunchKernelGGL(k_gather<false>, dim3(colblocks), dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st, pivx,
                       pivz, cols, SymCtx{});
  }
  return hipGetLastError();
}

hipError_t launch_rowsum(const TabDev &t, const u64 *mask, const u32 *cols, const MeasState *st, u64 *cnt0,
                         u64 *cnt1, u32 block, u32 wpt, u32 cpc, u32 max_chunks, const SymCtx *sym, hipStream_t s) {
  const u32 tiles = cdiv(t.L, (u64)block * wpt);
  const u32 vchunks = sym ? cdiv(sym->count, SIGN_COLS_PER_BLOCK) : 0;
  dim3 grid(tiles, max_chunks + vchunks);
  const SymCtx sc = sym ? *sym : SymCtx{};
  if (sym) {
    if (wpt == 2)
      hipLaunchKernelGGL((k_rowsum<2, 4, true>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1, t.Ls,
                         t.L, cpc, max_chunks, sc);
    else
      hipLaunchKernelGGL((k_rowsum<1, 4, true>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1, t.Ls,
                         t.L, cpc, max_chunks, sc);
  } else {
    if (wpt == 2)
      hipLaunchKernelGGL((k_rowsum<2, 4, false>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1,
                         t.Ls, t.L, cpc, max_chunks, sc);
    else
      hipLaunchKernelGGL((k_rowsum<1, 4, false>), grid, dim3(block), 0, s, t.X, t.Z, mask, cols, st, cnt0, cnt1,
                         t.Ls, t.L, cpc, max_chunks, sc);
  }
  return hipGetLastError();
}

hipError_t launch_post(const TabDev &t, const Cursor *cur, const u64 *mask, const u64 *pivx, const u64 *pivz,
                       const u64 *cnt0, const u64 *cnt1, const u32 *alist, MeasState *st, MeasStats *stats, u32 cpc,
                       u32 cpw, const SymCtx *sym, hipStream_t s) {
  // roles: a wave per sign word (4 per block), a thread per column, a block per
  // deterministic column range (and per affine-form word on the sampling path,
  // up to the last list position)
  u32 blocks = std::max(std::max(cdiv(t.L, 4), cdiv(t.n, 256)), cdiv(t.n, cpw));
  if (sym) blocks = std::max(blocks, cdiv(sym->count + 1, 64));
  if (sym)
    hipLaunchKernelGGL(k_post<true>, dim3(blocks), dim3(256), 0, s, t.X, t.Z, t.R, mask, pivx, pivz, cnt0, cnt1,
                       alist, st, stats, cur, t.Ls, t.L, t.K, t.n, cpc, cpw, *sym);
  else
    hipLaunchKernelGGL(k_post<false>, dim3(blocks), dim3(256), 0, s, t.X, t.Z, t.R, mask, pivx, pivz, cnt0, cnt1,
                       alist, st, stats, cur, t.Ls, t.L, t.K, t.n, cpc, cpw, SymCtx{});
  return hipGetLastError();
}

}  // namespace sq
