// Row-contiguous layout (the dual layout of "Tableau Layout and Indexing"):
// the in-place tile transpose of Algorithm alg:transpose, and CHP
// measurement kernels that work on whole generator rows.
//
// Row layout: slot r (the column slot r of the column layout, r < 64K, the
// X and Z blocks being allocated with 64K slots) holds generator pair r:
// words c < K the bits of D_r at qubits 64c .. 64c+63, words K + c those of
// S_r. Signs stay one per generator row (R is the same in both layouts).
// Each half (destabilizers, stabilizers) of X and of Z is a square bit
// matrix of 64K x 64K, so the transpose is the same operation both ways:
// every 64 x 64 bit tile (64 consecutive slots, one word) is transposed in
// registers and exchanged with its mirror tile.
//
// Measurement of Z_q in the row layout (one measurement per slot of kernels;
// "The CHP algorithm", both cases):
//   k_row_pivot   p = the smallest r with x_q(S_r) = 1 (word K + q/64 of
//                 each slot, a grid-wide minimum);
//   k_row_gather  the pivot row S_p copied out (contiguous), the coin;
//   k_row_rowsum  a wave per slot: each half with x_q = 1 (D_p and S_p
//                 excepted) becomes S_p times itself; the phase is a sum of
//                 per-word terms over the row, so each row costs its own
//                 words only (row-granular bytes);
//   k_row_det,    deterministic case: the product of the S_i with
//   k_row_det_combine   x_q(D_i) = 1, in ascending i, from the bilinear form
//                 of Pauli products: writing P = i^lam X^x Z^z,
//                 lam(P_1 ... P_m) = sum lam(P_i) + 2 sum_{i<i'} z_i . x_i'
//                 (mod 4); blocks of rows give partial sums and their XORs
//                 of x and z, and a second pass adds the cross terms of
//                 blocks (sum over b < b' of Zsum_b . Xsum_b');
//   k_row_finish  random: D_p <- S_p, S_p <- (-1)^coin Z_q; deterministic:
//                 the outcome; the cursor advances.
#include "sq_device.h"

namespace sq {

constexpr u32 TB = 16;         // tiles per side of a transposed block of tiles
constexpr u32 TLINE = TB + 1;  // LDS words per staged slot line (padded against bank conflicts)
constexpr u32 TLINES = 512;    // slot lines staged in LDS at a time (half a side)

// Grid (nb (nb + 1) / 2, 4): block (bi, bj), bi <= bj, of 16 x 16 tiles of
// one half of X or Z (y: matrix and half), processed with its mirror block
// (bj, bi); x enumerates the upper triangle row by row. A side is 1024 slots
// (64 per tile column) times 16 words: one 128-byte line per slot. Lines
// move between HBM and LDS coalesced, 512 at a time (70 KB of LDS, so two
// workgroups share a CU and overlap their phases); wave v holds slots
// 64 v .. 64 v + 63 of a side (a lane per slot, its 16 words in registers),
// transposes each tile in registers and writes it to its mirror position in
// LDS, from where the mirror side's lines are stored. Both sides are in
// registers before anything is stored, so a diagonal block is done in place
// by its own workgroup.
//
// Lines move 16 lanes per line, a word per lane: each wave instruction
// covers four whole 128-byte lines.
__device__ __forceinline__ void stage_in(const u64 *__restrict__ M, u64 *buf, u32 Ls, u32 K, u32 off, u32 slot0,
                                         u32 word0, u32 line0) {
  const u32 tid = threadIdx.x;
#pragma unroll
  for (u32 pass = 0; pass < TLINES / 64; ++pass) {
    const u32 line = pass * 64u + (tid >> 4), c = tid & 15u;
    const u32 slot = slot0 + line0 + line, w = word0 + c;
    const bool ok = (slot >> 6) < K && w < K;
    buf[line * TLINE + c] = ok ? __builtin_nontemporal_load(M + (size_t)slot * Ls + off + w) : 0ULL;
  }
}

__device__ __forceinline__ void stage_out(u64 *__restrict__ M, const u64 *buf, u32 Ls, u32 K, u32 off, u32 slot0,
                                          u32 word0, u32 line0) {
  const u32 tid = threadIdx.x;
#pragma unroll
  for (u32 pass = 0; pass < TLINES / 64; ++pass) {
    const u32 line = pass * 64u + (tid >> 4), c = tid & 15u;
    const u32 slot = slot0 + line0 + line, w = word0 + c;
    if ((slot >> 6) < K && w < K)
      __builtin_nontemporal_store(buf[line * TLINE + c], M + (size_t)slot * Ls + off + w);
  }
}

// One side into registers: lines [0, 512) then [512, 1024) through LDS.
__device__ __forceinline__ void side_in(const u64 *__restrict__ M, u64 *buf, u32 Ls, u32 K, u32 off, u32 slot0,
                                        u32 word0, u64 (&R)[TB]) {
  const u32 v = threadIdx.x >> 6, lane = threadIdx.x & 63u;
#pragma unroll
  for (u32 h = 0; h < 2; ++h) {
    stage_in(M, buf, Ls, K, off, slot0, word0, h * TLINES);
    __syncthreads();
    if ((v >> 3) == h) {
#pragma unroll
      for (u32 d = 0; d < TB; ++d) R[d] = buf[((v & 7u) * 64u + lane) * TLINE + d];
    }
    __syncthreads();
  }
}

// One side's transposed tiles out to the mirror side: tiles d < 8 fill the
// mirror's lines [0, 512), tiles d >= 8 its lines [512, 1024).
__device__ __forceinline__ void side_out(u64 *__restrict__ M, u64 *buf, u32 Ls, u32 K, u32 off, u32 slot0,
                                         u32 word0, const u64 (&R)[TB]) {
  const u32 v = threadIdx.x >> 6, lane = threadIdx.x & 63u;
#pragma unroll
  for (u32 h = 0; h < 2; ++h) {
#pragma unroll
    for (u32 d = 0; d < TB / 2; ++d) buf[(d * 64u + lane) * TLINE + v] = transpose64(R[h * (TB / 2) + d]);
    __syncthreads();
    stage_out(M, buf, Ls, K, off, slot0, word0, h * TLINES);
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_transpose(u64 *__restrict__ X, u64 *__restrict__ Z, u32 Ls, u32 K, u32 nb) {
  __shared__ u64 buf[TLINES * TLINE];
  // row bi of the triangle starts at bi nb - bi (bi - 1) / 2
  const u32 t = blockIdx.x;
  u32 bi = (u32)(((double)(2 * nb + 1) - sqrt((double)(2 * nb + 1) * (2 * nb + 1) - 8.0 * t)) * 0.5);
  auto row0 = [&](u32 r) { return r * nb - r * (r - 1) / 2; };
  while (bi > 0 && row0(bi) > t) --bi;
  while (row0(bi + 1) <= t) ++bi;
  const u32 bj = bi + (t - row0(bi));
  u64 *M = (blockIdx.y >> 1) ? Z : X;
  const u32 off = (blockIdx.y & 1u) ? K : 0u;
  // The stabilizer half starts at word K: its tile grid is shifted back by
  // K mod 16 tiles in both directions (a transpose keeps a symmetric grid),
  // so that every 16-word slot segment it moves starts on a 128-byte line.
  // Tiles before the first (negative indices, which wrap around in u32)
  // fail the range checks of the staging loops.
  const u32 sh = (blockIdx.y & 1u) ? (K & 15u) : 0u;
  const bool diag = bi == bj;
  const u32 slotA = 64u * (TB * bi - sh), wordA = TB * bj - sh;  // side A: its slots hold words wordA ..
  const u32 slotB = 64u * (TB * bj - sh), wordB = TB * bi - sh;  // the mirror side
  u64 A[TB], B[TB];
  side_in(M, buf, Ls, K, off, slotA, wordA, A);
  if (!diag) side_in(M, buf, Ls, K, off, slotB, wordB, B);
  // tile (16 bi + v, 16 bj + d) of side A becomes, lane j, slot 64 (16 bj + d) + j of side B at word 16 bi + v
  side_out(M, buf, Ls, K, off, slotB, wordB, A);
  if (!diag) side_out(M, buf, Ls, K, off, slotA, wordA, B);
}

// The pivot candidate starts at "none" (k_row_gather resets it after use).
__global__ void k_row_begin(MeasState *st) {
  if (threadIdx.x == 0) st->pc = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_row_pivot(const u64 *__restrict__ X, u32 Ls, u32 K, u32 n,
                                                   const Cursor *__restrict__ cur, MeasState *__restrict__ st) {
  const u32 i = cur->i;
  if (i >= cur->end) return;
  const u32 q = cur->qubits[i];
  const u32 wq = K + (q >> 6), sh = q & 63u;
  u32 first = 0xFFFFFFFFu;
  for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    if ((X[(size_t)r * Ls + wq] >> sh) & 1ULL) {
      first = r;
      break;
    }
  for (int off = 32; off > 0; off >>= 1) first = min(first, (u32)__shfl_xor((int)first, off));
  if ((threadIdx.x & 63u) == 0 && first != 0xFFFFFFFFu) atomicMin(&st->pc, first);
}

// One workgroup: the slot's measurement state, the coin, and (random case)
// the pivot row S_p copied to pivx/pivz with its count of nonzero words.
__global__ __launch_bounds__(1024) void k_row_gather(const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                                     const u64 *__restrict__ R, u32 Ls, u32 K,
                                                     Cursor *__restrict__ cur, MeasState *__restrict__ st,
                                                     u64 *__restrict__ pivx, u64 *__restrict__ pivz) {
  __shared__ int32_t s_p;
  __shared__ u32 s_nx, s_nz;
  const u32 tid = threadIdx.x;
  if (tid == 0) {
    const u32 i = cur->i;
    const u32 pc = st->pc;
    st->pc = 0xFFFFFFFFu;
    s_nx = s_nz = 0;
    if (i >= cur->end) {
      st->p = P_NONE;
      s_p = P_NONE;
    } else {
      const u32 q = cur->qubits[i];
      const int32_t p = pc == 0xFFFFFFFFu ? -1 : (int32_t)pc;
      const u32 c = coin_bit(cur->seed, cur->shot, cur->meas_base + i);
      st->p = p;
      st->q = q;
      st->i = i;
      st->coin = c;
      st->det_acc = 0;
      st->naff = 0;
      st->awords = 0;
      st->rp = p >= 0 ? (u32)(R[K + ((u32)p >> 6)] >> ((u32)p & 63u)) & 1u : 0u;
      if (cur->out_rand) cur->out_rand[i] = (uint8_t)(p >= 0);
      if (p >= 0 && cur->out_bits) cur->out_bits[i] = (uint8_t)c;
      s_p = p;
    }
  }
  __syncthreads();
  const int32_t p = s_p;
  if (p < 0) return;
  const u64 *xs = X + (size_t)p * Ls + K, *zs = Z + (size_t)p * Ls + K;
  u32 nx = 0, nz = 0;
  for (u32 c = tid; c < K; c += blockDim.x) {
    const u64 x = xs[c], z = zs[c];
    pivx[c] = x;
    pivz[c] = z;
    nx += x != 0;
    nz += z != 0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    nx += (u32)__shfl_xor((int)nx, off);
    nz += (u32)__shfl_xor((int)nz, off);
  }
  if ((tid & 63u) == 0) {
    atomicAdd(&s_nx, nx);
    atomicAdd(&s_nz, nz);
  }
  __syncthreads();
  if (tid == 0) {
    st->nx = s_nx;
    st->nz = s_nz;
  }
}

__device__ __forceinline__ u32 word_phase(u64 px, u64 pz, u64 qx, u64 qz) {
  return (u32)__popcll(px & pz) + (u32)__popcll(qx & qz) + 2u * (u32)__popcll(pz & qx) -
         (u32)__popcll((px ^ qx) & (pz ^ qz));
}

// A wave per slot r: each half (D_r, S_r) with x_q = 1, other than D_p and
// S_p, becomes S_p times itself: x ^= x_p, z ^= z_p (stored only where the
// pivot word is nonzero) and r <- (2 r + 2 r_p + phase) / 2, the phase of
// S_p * row summed over the row's words (must be even, else flag bit 0).
// The affected halves are walked as one run of words (both halves of a
// slot are contiguous), four rounds of loads in flight per lane; with
// LDS = true the workgroup first stages the pivot row (2K words) in LDS.
constexpr u32 ROWSUM_T = 1024;
constexpr u32 ROWSUM_LDS_MAX_K = 4096;  // 64 KB of pivot row

template <bool LDS>
__global__ __launch_bounds__(ROWSUM_T) void k_row_rowsum(u64 *__restrict__ X, u64 *__restrict__ Z,
                                                         u64 *__restrict__ R, u32 Ls, u32 K, u32 n,
                                                         MeasState *__restrict__ st, const u64 *__restrict__ pivx,
                                                         const u64 *__restrict__ pivz) {
  extern __shared__ u64 spiv[];
  const int32_t p = st->p;
  if (p < 0) return;  // the same for every workgroup
  if constexpr (LDS) {
    for (u32 c = threadIdx.x; c < K; c += blockDim.x) {
      spiv[c] = pivx[c];
      spiv[K + c] = pivz[c];
    }
    __syncthreads();
  }
  const u32 lane = threadIdx.x & 63u;
  const u32 r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= n || r == (u32)p) return;  // uniform over the wave; no barriers below (D_p, S_p skipped)
  const u32 q = st->q, wq = q >> 6, sh = q & 63u, rp = st->rp;
  const size_t base = (size_t)r * Ls;
  const bool aD = (X[base + wq] >> sh) & 1ULL, aS = (X[base + K + wq] >> sh) & 1ULL;
  if (!aD && !aS) return;
  // words [c0, c1) of the slot change; the walk goes in 16-byte pairs from
  // the even word below c0 (a word outside [c0, c1) is stored back as read:
  // the wave owns the slot)
  const u32 c0 = aD ? 0u : K, c1 = aS ? 2u * K : K;
  u32 phD = 0, phS = 0;
#pragma unroll 2
  for (u32 c = (c0 & ~1u) + 2u * lane; c < c1; c += 128u) {
    const u64x2 xv = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(X + base + c));
    const u64x2 zv = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(Z + base + c));
    u64 xo[2] = {xv.x, xv.y}, zo[2] = {zv.x, zv.y};
    bool any = false;
#pragma unroll
    for (u32 h = 0; h < 2; ++h) {
      const u32 cc = c + h;
      if (cc < c0 || cc >= c1) continue;
      const u32 cw = cc < K ? cc : cc - K;
      u64 px, pz;
      if constexpr (LDS) {
        px = spiv[cw];
        pz = spiv[K + cw];
      } else {
        px = pivx[cw];
        pz = pivz[cw];
      }
      const u32 ph = word_phase(px, pz, xo[h], zo[h]);
      if (cc < K) phD += ph;
      else phS += ph;
      xo[h] ^= px;
      zo[h] ^= pz;
      any |= (px | pz) != 0;
    }
    if (any) {
      u64x2 xw, zw;
      xw.x = xo[0];
      xw.y = xo[1];
      zw.x = zo[0];
      zw.y = zo[1];
      __builtin_nontemporal_store(xw, reinterpret_cast<u64x2 *>(X + base + c));
      __builtin_nontemporal_store(zw, reinterpret_cast<u64x2 *>(Z + base + c));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    phD += (u32)__shfl_xor((int)phD, off);
    phS += (u32)__shfl_xor((int)phS, off);
  }
  if (lane == 0) {
#pragma unroll
    for (u32 h = 0; h < 2; ++h) {
      if (!(h ? aS : aD)) continue;
      u64 *rw = R + h * K + (r >> 6);
      const u32 rh = (u32)(*rw >> (r & 63u)) & 1u;
      const u32 e = (2u * rh + 2u * rp + (h ? phS : phD)) & 3u;
      if (e & 1u) atomicOr(&st->flags, 1u);
      if ((e >> 1) != rh) atomicXor(rw, 1ULL << (r & 63u));
    }
    atomicAdd(&st->naff, (u32)aD + (u32)aS);
  }
}

// Deterministic case, grid (row blocks, word ranges of 64): a wave walks the
// rows of its block in order, over its 64 words; rows with x_q(D_i) = 1
// contribute lam(S_i) = 2 r_i + |x_i & z_i| and the in-block pair terms
// z_{<i} . x_i (z_{<i} the XOR of the block's earlier rows), and the block's
// XORs of x and z go to xsum/zsum (row b of stride Ls) for the combine.
__global__ __launch_bounds__(64) void k_row_det(const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                                const u64 *__restrict__ R, u32 Ls, u32 K, u32 n, u32 rows_per,
                                                MeasState *__restrict__ st, u64 *__restrict__ xsum,
                                                u64 *__restrict__ zsum) {
  if (st->p != -1) return;
  const u32 lane = threadIdx.x & 63u;
  const u32 b = blockIdx.x, c = blockIdx.y * 64u + lane;
  const u32 q = st->q, wq = q >> 6, sh = q & 63u;
  const u32 r0 = b * rows_per, r1 = min(r0 + rows_per, n);
  u64 zp = 0, xs = 0;
  u32 acc = 0, na = 0;
  for (u32 r = r0; r < r1; r += 64) {
    // which of the next 64 rows are in the product (one load per lane), and
    // their signs (counted once, by the first word range)
    const u32 i = r + lane;
    const u32 in = i < r1 ? (u32)(X[(size_t)i * Ls + wq] >> sh) & 1u : 0u;
    if (in && blockIdx.y == 0) acc += 2u * ((u32)(R[K + (i >> 6)] >> (i & 63u)) & 1u);
    u64 m = __ballot(in);
    na += (u32)__popcll(m);
    while (m) {  // uniform
      const u32 j = (u32)__builtin_ctzll(m);
      m &= m - 1;
      const size_t base = (size_t)(r + j) * Ls + K;
      u64 x = 0, z = 0;
      if (c < K) {
        x = __builtin_nontemporal_load(X + base + c);
        z = __builtin_nontemporal_load(Z + base + c);
      }
      acc += 2u * (u32)__popcll(zp & x) + (u32)__popcll(x & z);
      zp ^= z;
      xs ^= x;
    }
  }
  if (c < K) {
    xsum[(size_t)b * Ls + c] = xs;
    zsum[(size_t)b * Ls + c] = zp;
  }
  for (int off = 32; off > 0; off >>= 1) acc += (u32)__shfl_xor((int)acc, off);
  if (lane == 0) {
    atomicAdd(&st->det_acc, acc);
    if (blockIdx.y == 0 && na) atomicAdd(&st->awords, na);
  }
}

// Cross terms of the blocks, a wave per word range: sum over b' of
// (XOR of zsum_b, b < b') . xsum_b'.
__global__ __launch_bounds__(64) void k_row_det_combine(u32 Ls, u32 K, u32 nblocks, MeasState *__restrict__ st,
                                                        const u64 *__restrict__ xsum, const u64 *__restrict__ zsum) {
  if (st->p != -1) return;
  const u32 lane = threadIdx.x & 63u, c = blockIdx.x * 64u + lane;
  u64 zr = 0;
  u32 acc = 0;
  if (c < K)
    for (u32 b = 0; b < nblocks; ++b) {
      acc += 2u * (u32)__popcll(zr & xsum[(size_t)b * Ls + c]);
      zr ^= zsum[(size_t)b * Ls + c];
    }
  for (int off = 32; off > 0; off >>= 1) acc += (u32)__shfl_xor((int)acc, off);
  if (lane == 0 && acc) atomicAdd(&st->det_acc, acc);
}

// One workgroup. Random: D_p <- S_p (the copy in pivx/pivz), S_p <- Z_q with
// sign = coin. Deterministic: the outcome is half the phase exponent of the
// product (which is +-Z_q, so the exponent must be even: flag bit 1 else).
// Then the byte counts, and the cursor moves on.
__global__ __launch_bounds__(1024) void k_row_finish(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ R,
                                                     u32 Ls, u32 K, Cursor *__restrict__ cur,
                                                     MeasState *__restrict__ st, const u64 *__restrict__ pivx,
                                                     const u64 *__restrict__ pivz, MeasStats *__restrict__ stats) {
  const int32_t p = st->p;
  if (p == P_NONE) return;
  const u32 tid = threadIdx.x, q = st->q;
  if (p >= 0) {
    u64 *xr = X + (size_t)p * Ls, *zr = Z + (size_t)p * Ls;
    for (u32 c = tid; c < K; c += blockDim.x) {
      xr[c] = pivx[c];
      zr[c] = pivz[c];
      xr[K + c] = 0;
      zr[K + c] = (c == (q >> 6)) ? (1ULL << (q & 63u)) : 0ULL;
    }
  }
  if (tid == 0) {
    const u32 i = st->i;
    if (p >= 0) {
      const u64 bit = 1ULL << ((u32)p & 63u);
      u64 *rd = R + ((u32)p >> 6), *rs = R + K + ((u32)p >> 6);
      const u32 dnow = (u32)(*rd >> ((u32)p & 63u)) & 1u, snow = (u32)(*rs >> ((u32)p & 63u)) & 1u;
      if (dnow != st->rp) atomicXor(rd, bit);
      if (snow != st->coin) atomicXor(rs, bit);
      stats->n_random += 1;
      stats->rowsum_bytes += (u64)st->naff * 8ull * (2ull * K + st->nx + st->nz);
    } else {
      const u32 acc = st->det_acc;
      if (acc & 1u) atomicOr(&st->flags, 2u);
      if (cur->out_bits) cur->out_bits[i] = (uint8_t)((acc >> 1) & 1u);
      stats->n_det += 1;
      stats->det_bytes += (u64)st->awords * 16ull * K;
    }
    cur->i = i + 1;
  }
}

// Launchers.
hipError_t launch_transpose(const TabDev &t, hipStream_t s) {
  const u32 nb = cdiv(t.K + (t.K & 15u), TB);  // blocks per side, room for the shifted grid
  hipLaunchKernelGGL(k_transpose, dim3(nb * (nb + 1) / 2, 4), dim3(1024), 0, s, t.X, t.Z, t.Ls, t.K, nb);
  return hipGetLastError();
}

hipError_t launch_row_begin(MeasState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_row_begin, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_row_prep(const TabDev &t, Cursor *cur, MeasState *st, u64 *pivx, u64 *pivz, hipStream_t s) {
  const u32 pivot_blocks = std::min<u32>(cdiv(t.n, 256), 1024);
  hipLaunchKernelGGL(k_row_pivot, dim3(pivot_blocks), dim3(256), 0, s, t.X, t.Ls, t.K, t.n, cur, st);
  hipLaunchKernelGGL(k_row_gather, dim3(1), dim3(1024), 0, s, t.X, t.Z, t.R, t.Ls, t.K, cur, st, pivx, pivz);
  return hipGetLastError();
}

hipError_t launch_row_rowsum(const TabDev &t, MeasState *st, const u64 *pivx, const u64 *pivz, hipStream_t s) {
  const dim3 grid(cdiv(t.n, ROWSUM_T / 64)), block(ROWSUM_T);
  if (t.K <= ROWSUM_LDS_MAX_K)
    hipLaunchKernelGGL(k_row_rowsum<true>, grid, block, (size_t)2 * t.K * 8, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st,
                       pivx, pivz);
  else
    hipLaunchKernelGGL(k_row_rowsum<false>, grid, block, 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st, pivx, pivz);
  return hipGetLastError();
}

// det_blocks row blocks (their partial XORs are rows of xsum/zsum).
hipError_t launch_row_det(const TabDev &t, MeasState *st, u64 *xsum, u64 *zsum, u32 det_blocks, hipStream_t s) {
  const u32 rows_per = cdiv(t.n, det_blocks), nb = cdiv(t.n, rows_per), nc = cdiv(t.K, 64);
  hipLaunchKernelGGL(k_row_det, dim3(nb, nc), dim3(64), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, rows_per, st, xsum,
                     zsum);
  hipLaunchKernelGGL(k_row_det_combine, dim3(nc), dim3(64), 0, s, t.Ls, t.K, nb, st, xsum, zsum);
  return hipGetLastError();
}

hipError_t launch_row_finish(const TabDev &t, Cursor *cur, MeasState *st, const u64 *pivx, const u64 *pivz,
                             MeasStats *stats, hipStream_t s) {
  hipLaunchKernelGGL(k_row_finish, dim3(1), dim3(1024), 0, s, t.X, t.Z, t.R, t.Ls, t.K, cur, st, pivx, pivz, stats);
  return hipGetLastError();
}

}  // namespace sq
