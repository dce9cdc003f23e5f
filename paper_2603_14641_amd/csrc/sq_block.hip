// Blocked random measurements: up to KB consecutive random Z measurements
// applied in one streaming pass over the tableau, bit-identical to applying
// them one by one with CHP.
//
// Let measurements s = 0..k-1 measure q_s with pivots P_s = S_{p_s} as they
// stand just before measurement s. A row h that is not D_{p_s} or S_{p_s} of
// any s ends as C_h h with C_h = P_{s_m} ... P_{s_1} (the pivots that hit it,
// in order). Whether pivot s hits h is linear over GF(2) in h's bits at the
// measured columns: b_s = a_s ^ XOR_{s'<s} b_{s'} M[s'][s], where a_s is h's x
// bit at q_s before the block and M[s'][s] is P_{s'}'s x bit at q_s. The x/z
// update is then XOR_s b_s P_s. Signs follow from writing a Pauli as
// i^lam X^x Z^z with lam = 2 r + |x & z| (mod 4), in which products are
// bilinear: lam(A B) = lam(A) + lam(B) + 2 (z_A . x_B). So
//   lam(C_h h) = sum_s b_s lam(P_s) + 2 sum_{s<s'} b_s b_s' (z_{P_s'} . x_{P_s})
//                + lam(h) + 2 XOR_s b_s (z_{P_s} . x_h)   (mod 4),
// and the new sign is (lam - |x' & z'|) / 2, the difference being even. The
// last term is z_{C_h} . x_h, and per column j the bit z_{C_h}(j) =
// XOR_s b_s z_{P_s}(j) is exactly the z update the pass applies there, so it
// is the XOR over columns of (z update & x). Per row word the pass keeps
// |x & z| - |x' & z'| (mod 4, over columns where some pivot is not the
// identity) as a 2-bit counter and that one parity word. D_{p_s} becomes P_s times the later
// pivots that hit it; S_{p_s} becomes (-1)^coin Z_{q_s}. The block ends before
// the first deterministic measurement, which then takes the single path.
#include "sq_device.h"

namespace sq {

// -------------------------------------------------------------- pivots (one workgroup)
// Sequential over the measurements of the block; within a step the
// stabilizer words are spread over the workgroup's waves. For step s the
// stabilizer half of column q_s as it stands before measurement s is
//   X_{q_s} ^ XOR_{s' < s, M[s'][s] = 1} (hit mask of s'),
// with X as it stands before the block (nothing writes X until the pass) and
// the rows S_{p_s'} (now Z_{q_s'}, no x) cleared. Unrolled, that sum is a
// fixed GF(2) combination of the block's columns: with C = (I + M)^-1 (upper
// triangular, column s = e_s plus the columns s' < s with M[s'][s] = 1),
// step s's word is XOR_{t: C[t][s] = 1} X_{q_t}, earlier pivot rows cleared
// (a cleared bit stays cleared through every later sum). The tiled search
// computes any word of any step straight from the columns; the register
// search keeps the rows themselves. Words come in tiles of 64; wave v owns
// the tiles t = v mod (waves) and lane l word 64t + l; each wave walks its
// tiles in order and stops at its first nonzero tile; the smallest such
// word over the waves holds the pivot. A block ends before its first
// deterministic measurement (no nonzero word).
// The lane that owns the pivot word does the step's bookkeeping, so a step
// costs two barriers; the per-pivot outputs are written once at the end.
constexpr u32 PW_WAVES = 8;

// The block's measurements: list[i0 .. i0 + want) from the cursor, want =
// min(kb, end - i0), 0 once the list is done. Thread 0 reads the cursor and
// the qubits into LDS; every thread returns with the values.
__device__ __forceinline__ void block_take(const Cursor *__restrict__ cur, u32 *sq, u32 *s_hdr, u32 &i0, u32 &want) {
  if (threadIdx.x == 0) {
    const u32 i = cur->i, end = cur->end;
    const u32 w = i < end ? min(cur->kb, end - i) : 0u;
    s_hdr[0] = i;
    s_hdr[1] = w;
  }
  __syncthreads();
  i0 = s_hdr[0];
  want = s_hdr[1];
  if (threadIdx.x < KB) sq[threadIdx.x] = threadIdx.x < want ? cur->qubits[i0 + threadIdx.x] : 0u;
  __syncthreads();
}

// The per-pivot outputs of a block, by wave 0 of the pivot kernels (lane s
// for pivot s): positions, qubits, hit sets, M, the coins and outcome bytes,
// the later pivots that hit each D_{p_s}, zeroed sums for the pivot algebra,
// and the pivots grouped by row word. Lane 0 then advances the cursor past the
// block and flags the deterministic measurement that ended it (if any) for the
// slot's single kernels.
__device__ void pivots_finish(u32 lane, u32 k, u32 want, u32 i0, const u32 *sq, const u32 *piv, const u32 *mrow,
                              const u32 *mcol, const u32 *hits, Cursor *__restrict__ cur, BlkState *__restrict__ bs) {
  const u32 s = lane;
  const bool on = s < k;
  if (s < KB) bs->q[s] = sq[s];
  if (on) {
    const u32 c = coin_bit(cur->seed, cur->shot, cur->meas_base + i0 + s);
    bs->p[s] = piv[s];
    bs->hitS[s] = hits[s];
    bs->M[s] = mrow[s];
    bs->coin[s] = c;
    if (cur->out_rand) cur->out_rand[i0 + s] = 1;
    if (cur->out_bits) cur->out_bits[i0 + s] = (uint8_t)c;
    // later pivots that hit D_{p_s} (which holds P_s from measurement s on)
    u32 h = 0;
    for (u32 s2 = s + 1; s2 < k; ++s2) h |= (((mrow[s] >> s2) ^ (u32)__popc(h & mcol[s2])) & 1u) << s2;
    bs->dhits[s] = h;
  }
  if (s < KB) {
    bs->Qz[s] = 0;
    bs->R0[s] = 0;
    bs->pc0[s] = 0;
    bs->pcD[s] = 0;
  }
  // group the pivots by row word (pivots of a block usually share one or two),
  // words numbered in order of first use
  const u32 wd = on ? piv[s] >> 6 : 0xFFFFFFFFu;
  u32 same = 0;  // pivots on this lane's word
  for (u32 s2 = 0; s2 < k; ++s2) same |= ((u32)__shfl((int)wd, (int)s2) == wd ? 1u : 0u) << s2;
  const bool first = on && (same & ((1u << s) - 1u)) == 0;
  const u64 fb = __ballot(first);
  if (first) {
    const u32 i = (u32)__popcll(fb & ((1ULL << s) - 1ULL));
    bs->word[i] = wd;
    bs->wmem[i] = same;
  }
  if (lane == 0) {
    bs->k = k;
    bs->i0 = i0;
    bs->nwords = (u32)__popcll(fb);
    bs->ncols = 0;
    cur->i = i0 + k;
    cur->single = k < want ? 1u : 0u;
  }
}


// Before the tiled search: where each measured column's stabilizer half
// starts to be nonzero. Grid (cdiv(K, 256), KB): workgroup (g, s) writes the
// first stabilizer word in [256 g, 256 g + 256) where column q_s of X is
// nonzero (0xFFFFFFFF for none) to fz[s * G + g], for the s < want of the
// block the cursor offers. Step s of the search then starts at
//   lb_s = min over s' <= s of (column q_s' first nonzero word):
// below lb_s the column and every earlier step's row (a sum of hit rows of
// the earlier columns) are zero, so those tiles need no visit.
__global__ __launch_bounds__(256) void k_blk_firstnz(const u64 *__restrict__ X, u32 Ls, u32 K,
                                                     const Cursor *__restrict__ cur, u32 *__restrict__ fz, u32 G) {
  __shared__ u32 s_min;
  const u32 s = blockIdx.y, g = blockIdx.x, tid = threadIdx.x;
  const u32 i = cur->i, end = cur->end;
  const u32 want = i < end ? min(cur->kb, end - i) : 0u;
  if (s >= want) return;  // uniform over the workgroup
  const u32 q = cur->qubits[i + s];
  if (tid == 0) s_min = 0xFFFFFFFFu;
  __syncthreads();
  const u32 w = g * 256u + tid;
  const bool nz = w < K && X[(size_t)q * Ls + K + w] != 0ULL;
  const u64 b = __ballot(nz);
  if (b && (tid & 63u) == 0) atomicMin(&s_min, g * 256u + (tid & ~63u) + (u32)__builtin_ctzll(b));
  __syncthreads();
  if (tid == 0) fz[s * G + g] = s_min;
}

__global__ __launch_bounds__(64 * PW_WAVES) void k_blk_pivots(const u64 *__restrict__ X, u32 Ls, u32 K,
                                                               Cursor *__restrict__ cur, BlkState *__restrict__ bs,
                                                               u64 *__restrict__ zw, u32 nzw,
                                                               const u32 *__restrict__ fz, u32 G) {
  __shared__ u32 s_wmin[2];  // double-buffered: step s uses s_wmin[s & 1]
  // per-step state in LDS (indexed by step, which is not a compile-time
  // constant)
  __shared__ u32 piv[KB];   // pivot of each decided step
  __shared__ u32 mrow[KB];  // M[s]: bit s2 = x of P_s at q_{s2}
  __shared__ u32 mcol[KB];  // bit s' of mcol[s] = M[s'][s]
  __shared__ u32 hits[KB];  // earlier pivots that hit S_{p_s}
  __shared__ u32 ccol[KB];  // bit t of ccol[s] = C[t][s]: row s is the sum of the columns q_t in it
  __shared__ u32 sq[KB];    // measured qubits (step s reads column q_s of X)
  __shared__ u32 s_hdr[2];
  __shared__ u32 slb[KB];   // lb_s: below this word step s's row is zero
  const u32 tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwv = blockDim.x >> 6;
  const u32 ntiles = (K + 63u) / 64u;
  if (tid < KB) { piv[tid] = 0; mrow[tid] = 0; mcol[tid] = 0; hits[tid] = 0; ccol[tid] = 0; }
  if (tid < 2) s_wmin[tid] = 0xFFFFFFFFu;
  for (u32 i = tid; i < nzw; i += blockDim.x) zw[i] = 0;  // words the slot's later kernels need zeroed
  u32 i0, want;
  block_take(cur, sq, s_hdr, i0, want);
  // each column's first nonzero stabilizer word: 32 threads per step, a
  // minimum over the chunks, then the prefix minimum over the steps
  for (u32 s = tid >> 5; s < KB; s += blockDim.x >> 5) {
    u32 m = 0xFFFFFFFFu;
    if (s < want)
      for (u32 g = tid & 31u; g < G; g += 32u) m = min(m, fz[s * G + g]);
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) m = min(m, (u32)__shfl_xor((int)m, off));
    if ((tid & 31u) == 0) slb[s] = m;
  }
  __syncthreads();
  if (tid == 0)
    for (u32 s = 1; s < want; ++s) slb[s] = min(slb[s], slb[s - 1]);
  __syncthreads();
  // this wave's first tile at or past word lb (local tile j is tile j nwv + wave)
  auto first_tile = [&](u32 lb) -> u32 {
    const u32 t = lb >> 6;
    return t <= wave ? 0u : (t - wave + nwv - 1u) / nwv;
  };
  auto word_of = [&](u32 j) { return (j * nwv + wave) * 64u + lane; };  // local tile j
  // Row s at word w: the columns q_t with bit t of c (C[t][s]) summed, the
  // earlier pivot rows cleared. Every column is loaded (the ones not in c
  // are masked), so the loads are independent and in flight together.
  auto tile_word = [&](u32 s, u32 c, u32 w) -> u64 {
    if (w >= K) return 0ULL;
    u64 b[KB];
#pragma unroll
    for (u32 t = 0; t < KB; ++t) b[t] = X[(size_t)sq[t] * Ls + K + w];  // past want: column q_0's word
    u64 v = 0;
#pragma unroll
    for (u32 t = 0; t < KB; ++t) v ^= ((c >> t) & 1u) ? b[t] : 0ULL;
#pragma unroll
    for (u32 sp = 0; sp < KB; ++sp) {
      const u32 pv = piv[sp];
      if (sp < s && (pv >> 6) == w) v &= ~(1ULL << (pv & 63u));  // S_{p_s'} is Z now
    }
    return v;
  };
  const u32 myt = ntiles > wave ? (ntiles - wave + nwv - 1) / nwv : 0;  // tiles of this wave
  u32 k = want;
  for (u32 s = 0; s < want; ++s) {
    // C's column s: step s's own column plus the columns of the earlier rows
    // that hit it (M[s'][s] of every s' < s is known)
    u32 c = 1u << s;
    for (u32 m = mcol[s]; m != 0u; m &= m - 1u) c ^= ccol[__builtin_ctz(m)];
    if (tid == 0) ccol[s] = c;  // read by later steps, after this step's barriers
    u64 vlast = 0;  // this lane's word of step s in the last tile the wave computed
    for (u32 j = first_tile(slb[s]); j < myt; ++j) {
      const u32 w = word_of(j);
      const u64 v = tile_word(s, c, w);
      vlast = v;
      const u64 nz = __ballot(v != 0);
      if (nz) {  // uniform over the wave
        if (lane == (u32)__builtin_ctzll(nz)) atomicMin(&s_wmin[s & 1u], w);
        break;
      }
    }
    __syncthreads();
    const u32 wmin = s_wmin[s & 1u];
    if (wmin == 0xFFFFFFFFu) {  // deterministic: the block ends here
      k = s;
      break;
    }
    if (tid == 0) s_wmin[(s + 1) & 1u] = 0xFFFFFFFFu;  // its last reader passed the barrier above
    // the owning wave (the one whose last tile holds word wmin) does the
    // step's bookkeeping, one lane per step
    if (wave == (wmin >> 6) % nwv) {
      const u32 pl = wmin & 63u;
      const u32 pb = (u32)__builtin_ctzll(shfl_u64(vlast, (int)pl));
      // every measured column of X at word wmin; bit t of xb: column q_t has
      // x at row p
      const u64 sv = lane < want ? X[(size_t)sq[lane] * Ls + K + wmin] : 0ULL;
      const u32 xb = (u32)__ballot(((sv >> pb) & 1ULL) != 0);
      // earlier pivots that hit S_p: row s' has x at p (p is none of the
      // earlier pivots, so the cleared bits do not matter there)
      const bool h = lane < s && (__popc(ccol[lane & (KB - 1u)] & xb) & 1);
      const u32 hit = (u32)__ballot(h);
      // x bit of P_s at the later measured column q_lane: X's bit at p plus
      // the earlier pivots that hit S_p (M is known for those)
      const bool later = lane > s && lane < want;
      const bool mine = later && ((((u32)(sv >> pb)) ^ (u32)__popc(hit & mcol[lane & (KB - 1u)])) & 1u);
      const u32 mb = (u32)__ballot(mine);
      if (mine) mcol[lane] |= 1u << s;
      if (lane == 0) {
        piv[s] = wmin * 64u + pb;
        mrow[s] = mb;
        hits[s] = hit;
      }
    }
    __syncthreads();
  }
  if (wave == 0) pivots_finish(lane, k, want, i0, sq, piv, mrow, mcol, hits, cur, bs);
}

// Small tableaux (at most PR_WAVES tiles of 64 stabilizer words): lane l
// owns word l and keeps its rows of every step and its words of the
// measured columns in registers, so a step touches LDS only. Every word is evaluated at every
// step (the recurrence above, with the step loop unrolled so that rows are
// indexed by constants); the pivots already found in a lane's word are left
// out of its search, and the pivot's owner lane does the step's bookkeeping.
constexpr u32 PR_WAVES = 8;

__global__ __launch_bounds__(64 * PR_WAVES) void k_blk_pivots_reg(const u64 *__restrict__ X, u32 Ls, u32 K,
                                                                  Cursor *__restrict__ cur,
                                                                  BlkState *__restrict__ bs, u64 *__restrict__ zw,
                                                                  u32 nzw) {
  __shared__ u32 s_wmin[2];  // double-buffered: step s uses s_wmin[s & 1]
  __shared__ u32 piv[KB], mrow[KB], mcol[KB], hits[KB], sq[KB], s_hdr[2];
  const u32 tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const u32 w = tid;  // this lane's stabilizer word
  const bool in = w < K;
  if (tid < KB) { piv[tid] = 0; mrow[tid] = 0; mcol[tid] = 0; hits[tid] = 0; }
  if (tid < 2) s_wmin[tid] = 0xFFFFFFFFu;
  for (u32 i = tid; i < nzw; i += blockDim.x) zw[i] = 0;  // words the slot's later kernels need zeroed
  u32 i0, want;
  block_take(cur, sq, s_hdr, i0, want);
  u64 sn[KB], rv[KB];
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {  // steps past want are masked out below
    // every load issued (steps past want read column q_0 and are masked), so
    // that none waits behind a branch
    const u64 v = in ? X[(size_t)sq[s < want ? s : 0] * Ls + K + w] : 0ULL;
    sn[s] = s < want ? v : 0ULL;
    rv[s] = 0;
  }
  u64 spec = 0;  // pivots found in this word so far (rows S_{p_s'}: Z now, no x)
  const u32 kall = want >= KB ? 0xFFFFFFFFu : (1u << want) - 1u;
  u32 k = want;
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {
    if (s < k) {  // uniform
      const u32 sel = __builtin_amdgcn_readfirstlane(mcol[s]);  // M[s'][s] of the earlier steps
      u64 v = sn[s];
#pragma unroll
      for (u32 sp = 0; sp < s; ++sp) v = xor_and(v, rv[sp], 0u - ((sel >> sp) & 1u));
      rv[s] = v;
      const u64 vc = v & ~spec;
      const u64 nz = __ballot(vc != 0);
      if (nz && lane == (u32)__builtin_ctzll(nz)) atomicMin(&s_wmin[s & 1u], w);
      __syncthreads();
      const u32 wmin = s_wmin[s & 1u];
      if (wmin == 0xFFFFFFFFu) {  // deterministic: the block ends here
        k = s;
      } else {
        if (tid == 0) s_wmin[(s + 1) & 1u] = 0xFFFFFFFFu;  // its last reader passed the barrier above
        if (wave == (wmin >> 6)) {  // the owner wave; lane pl owns word wmin
          const u32 pl = wmin & 63u;
          const u32 pb = (u32)__builtin_ctzll(shfl_u64(vc, (int)pl));
          // every lane takes bit pb of its rows and measured columns; lane pl's
          // are row p's: the earlier pivots that hit S_p, and X's bits at p
          u32 hv = 0, sv = 0;
#pragma unroll
          for (u32 sp = 0; sp < s; ++sp) hv |= (u32)((rv[sp] >> pb) & 1ULL) << sp;
#pragma unroll
          for (u32 s2 = s + 1; s2 < KB; ++s2) sv |= (u32)((sn[s2] >> pb) & 1ULL) << s2;
          const u32 hit = (u32)__shfl((int)hv, (int)pl), snb = (u32)__shfl((int)sv, (int)pl);
          // lane s2 > s: x bit of P_s at q_{s2} (the earlier pivots that hit S_p
          // add their own, known for those)
          const bool mine = lane > s && ((kall >> (lane & 31u)) & 1u) && lane < KB &&
                            (((snb >> lane) ^ (u32)__popc(hit & mcol[lane & (KB - 1u)])) & 1u);
          const u32 mb = (u32)__ballot(mine);
          if (mine) mcol[lane] |= 1u << s;
          if (lane == pl) spec |= 1ULL << pb;
          if (lane == 0) {
            piv[s] = wmin * 64u + pb;
            mrow[s] = mb;
            hits[s] = hit;
          }
        }
        __syncthreads();
      }
    }
  }
  if (wave == 0) pivots_finish(lane, k, want, i0, sq, piv, mrow, mcol, hits, cur, bs);
}

// -------------------------------------------------------------- hit masks
// Thread per row word: bit h of mask s says pivot s multiplies row h. For
// every row outside the special ones the recurrence
//   b_s = a_s ^ XOR_{s' < s} b_{s'} M[s'][s]
// holds; the special rows (D_p and S_p of every pivot) take no part in the
// pass and are cleared.
__device__ __forceinline__ void blk_masks(const u64 *__restrict__ X, u64 *__restrict__ bm,
                                          const BlkState *__restrict__ bs, u32 Ls, u32 L, u32 K, u32 bid) {
  __shared__ u32 spv[KB], sq[KB];  // pivot rows, measured qubits
  const u32 k = bs->k;
  if (k == 0) return;  // the same for every workgroup
  if (threadIdx.x < KB) {  // entries past k are not read
    spv[threadIdx.x] = bs->p[threadIdx.x];
    sq[threadIdx.x] = bs->q[threadIdx.x];
  }
  __syncthreads();
  const u32 w = bid * blockDim.x + threadIdx.x;
  if (w >= L) return;
  u64 special = 0;
  const u32 hw = w < K ? w : w - K;
  for (u32 t = 0; t < k; ++t)
    if ((spv[t] >> 6) == hw) special |= 1ULL << (spv[t] & 63u);
  u64 b[KB];
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {  // all loads issued (past k: column q_0, masked)
    const u64 v = X[(size_t)sq[s < k ? s : 0] * Ls + w];
    b[s] = s < k ? v : 0ULL;
  }
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {
    if (s < k) {
#pragma unroll
      for (u32 sp = 0; sp < s; ++sp)
        if ((bs->M[sp] >> s) & 1u) b[s] ^= b[sp];
    }
  }
#pragma unroll
  for (u32 s = 0; s < KB; ++s)
    if (s < k) bm[(size_t)s * Ls + w] = b[s] & ~special;
}

// Distinct row words holding pivots whose loads a thread issues together
// (blk_special, blk_sv_prep).
constexpr u32 SPEC_B = 8;

// -------------------------------------------------------------- pivot rows and their algebra
// Grid cdiv(n, ROWS_T): thread per column j, wave per 64-column word cw.
// (1) The original pivot rows' bits at the wave's columns: one read of x and
// z per distinct stabilizer word holding pivots, a ballot per pivot.
// (2) The evolved pivot rows P_s = S0_{p_s} times the earlier pivots that hit
// it, in order (uniform over the wave). (3) The column patterns: bit s of
// patx[j] / patz[j] = P_s has x / z at j; columns where some P_s is not the
// identity are counted. (4) The word's share of the pair products, lane a
// for pivot a: bits b of z_{P_a} . x_{P_b} (Qz) and of z_{P_a} . x_{S0_b}
// (R0), |x & z| of the final D_{p_a} (P_a times its later hits) and of the
// original row S0_{p_a}, the counts mod 4; the block combines its waves'
// shares in LDS and writes one; blk_algebra then sums the blocks' shares
// and forms lam(P_s) and the final signs of the D_{p_s}.
constexpr u32 ROWS_T = 256;
constexpr u32 ROWS_W = ROWS_T / 64;  // waves per block

__device__ __forceinline__ void blk_rows(const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                         const u64 *__restrict__ R, u32 Ls, u32 K, u32 n, BlkState *__restrict__ bs,
                                         u32 *__restrict__ patx, u32 *__restrict__ patz, u32 *__restrict__ wpart,
                                         u32 *__restrict__ clist, u32 bid) {
  __shared__ u64 s0x[ROWS_W][KB], s0z[ROWS_W][KB], sx[ROWS_W][KB], sz[ROWS_W][KB];
  __shared__ u32 red[4][ROWS_T / KB][KB];  // per-wave shares
  const u32 k = bs->k;
  if (k == 0) return;  // the same for every workgroup
  const u32 tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const u32 j = bid * ROWS_T + tid;
  const u32 cw = j >> 6;  // uniform over the wave
  // (1) original rows, into LDS (rows past k stay zero)
  if (lane < KB) {
    s0x[wv][lane] = 0;
    s0z[wv][lane] = 0;
  }
  const u32 nw = bs->nwords;
  for (u32 i = 0; i < nw; ++i) {
    const u32 ws = K + bs->word[i], mem = bs->wmem[i];
    u64 xw = 0, zw = 0;
    if (j < n) {
      xw = X[(size_t)j * Ls + ws];
      zw = Z[(size_t)j * Ls + ws];
    }
#pragma unroll
    for (u32 s = 0; s < KB; ++s) {
      if ((mem >> s) & 1u) {  // uniform
        const u32 sh = bs->p[s] & 63u;
        const u64 bx = __ballot((xw >> sh) & 1u), bz = __ballot((zw >> sh) & 1u);
        if (lane == 0) {
          s0x[wv][s] = bx;
          s0z[wv][s] = bz;
        }
        if (j == 0) bs->r0[s] = (u32)(R[ws] >> sh) & 1u;
      }
    }
  }
  __syncthreads();
  // (2) evolved rows
  u64 vx[KB], vz[KB];
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {
    const u32 h = s < k ? bs->hitS[s] : 0u;
    u64 ax = s0x[wv][s], az = s0z[wv][s];
#pragma unroll
    for (u32 sp = 0; sp < s; ++sp) {
      const u64 m = 0ULL - (u64)((h >> sp) & 1u);
      ax ^= vx[sp] & m;
      az ^= vz[sp] & m;
    }
    vx[s] = ax;
    vz[s] = az;
  }
  // (3) patterns (rows past k are zero)
  u32 px = 0, pz = 0;
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {
    px |= (u32)((vx[s] >> lane) & 1ULL) << s;
    pz |= (u32)((vz[s] >> lane) & 1ULL) << s;
  }
  if (j < n) {
    patx[j] = px;
    patz[j] = pz;
  }
  // the supported columns, compacted into clist (any order: the pass sums
  // over columns)
  const bool sup = j < n && (px | pz) != 0;
  const u64 sb = __ballot(sup);
  u32 cbase = 0;
  if (lane == 0 && sb) cbase = atomicAdd(&bs->ncols, (u32)__popcll(sb));
  cbase = (u32)__shfl((int)cbase, 0);
  if (sup) clist[cbase + (u32)__popcll(sb & lanemask_lt())] = j;
  // (4) pair shares, lane a for pivot a
  if (lane == 0) {
#pragma unroll
    for (u32 s = 0; s < KB; ++s) {
      sx[wv][s] = vx[s];
      sz[wv][s] = vz[s];
    }
  }
  __syncthreads();
  if (lane < KB) {
    const u32 a = lane;
    const u64 za = sz[wv][a];
    u32 qz = 0, r0 = 0;
#pragma unroll
    for (u32 b = 0; b < KB; ++b) {
      qz |= ((u32)__popcll(za & sx[wv][b]) & 1u) << b;
      r0 |= ((u32)__popcll(za & s0x[wv][b]) & 1u) << b;
    }
    const u32 dh = a < k ? bs->dhits[a] : 0u;
    u64 dx = sx[wv][a], dz = za;
#pragma unroll
    for (u32 b = 0; b < KB; ++b) {
      const u64 m = 0ULL - (u64)((dh >> b) & 1u);
      dx ^= sx[wv][b] & m;
      dz ^= sz[wv][b] & m;
    }
    const bool live = cw < K;  // a wave past the last word adds nothing
    red[0][wv][a] = live ? qz : 0u;
    red[1][wv][a] = live ? r0 : 0u;
    red[2][wv][a] = live ? (u32)__popcll(dx & dz) & 3u : 0u;
    red[3][wv][a] = live ? (u32)__popcll(s0x[wv][a] & s0z[wv][a]) & 3u : 0u;
  }
  __syncthreads();
  if (tid < KB) {  // the block's share, its waves combined
    u32 q = 0, r = 0, d = 0, p0 = 0;
#pragma unroll
    for (u32 g = 0; g < ROWS_W; ++g) {
      q ^= red[0][g][tid];
      r ^= red[1][g][tid];
      d += red[2][g][tid];
      p0 += red[3][g][tid];
    }
    u32 *wp = wpart + (size_t)bid * 4u * KB;
    wp[tid] = q;
    wp[KB + tid] = r;
    wp[2 * KB + tid] = d;
    wp[3 * KB + tid] = p0;
  }
}

// The pivot algebra of a block, once its row workgroups have written their
// shares (one workgroup of ROWS_T threads in a later launch, the last one of
// k_blk_reduce's grid): sums over the shares, lam(P_s) and the final signs
// of the D_{p_s}. The kernel boundary orders the shares' writes before these
// reads, so the row workgroups need no fence.
__device__ __forceinline__ void blk_algebra(const u32 *__restrict__ wpart, BlkState *__restrict__ bs,
                                            MeasState *__restrict__ st, u32 nblocks) {
  __shared__ u32 red[4][ROWS_T / KB][KB];
  const u32 k = bs->k;
  if (k == 0) return;
  const u32 tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  // sums over the blocks' shares: thread t takes pivot t mod KB and the
  // blocks g, g + G, ... with g = t / KB, G = ROWS_T / KB groups
  {
    constexpr u32 G = ROWS_T / KB;
    const u32 a = tid & (KB - 1u), g = tid / KB;
    u32 q = 0, r = 0, d = 0, p0 = 0;
#pragma unroll 4
    for (u32 bl = g; bl < nblocks; bl += G) {
      const u32 *wp = wpart + (size_t)bl * 4u * KB;
      q ^= wp[a];
      r ^= wp[KB + a];
      d += wp[2 * KB + a];
      p0 += wp[3 * KB + a];
    }
    red[0][g][a] = q;
    red[1][g][a] = r;
    red[2][g][a] = d;
    red[3][g][a] = p0;
  }
  __syncthreads();
  if (wv != 0) return;
  const u32 s = lane;
  const bool on = s < k;
  u32 qs = 0, rs = 0, pd = 0, base = 0, hs = 0, dh = 0;
  if (on) {
    u32 p0 = 0;
#pragma unroll
    for (u32 g = 0; g < ROWS_T / KB; ++g) {
      qs ^= red[0][g][s];
      rs ^= red[1][g][s];
      pd += red[2][g][s];
      p0 += red[3][g][s];
    }
    base = 2u * bs->r0[s] + p0;
    hs = bs->hitS[s];
    dh = bs->dhits[s];
    bs->Qz[s] = qs;
  }
  // lam(P_t): the original row times the earlier pivots sp that hit it, in
  // order; each factor adds lam(P_sp) + 2 (z_{P_sp} . x of the partial
  // product), whose x is x_{S0_t} ^ XOR of the factors before sp
  u32 lam = 0;
  for (u32 t = 0; t < k; ++t) {
    const u32 ht = (u32)__shfl((int)hs, (int)t);
    u32 term = 0;
    if (s < t && ((ht >> s) & 1u)) {  // hits of t are earlier pivots
      const u32 par = ((rs >> t) ^ (u32)__popc(qs & ht & ((1u << s) - 1u))) & 1u;
      term = (lam + 2u * par) & 3u;
    }
    const u32 sum = (u32)__popcll(__ballot(term & 1u)) + 2u * (u32)__popcll(__ballot((term >> 1) & 1u));
    const u32 bt = (u32)__shfl((int)base, (int)t);
    if (s == t) lam = (bt + sum) & 3u;
  }
  // final signs of the D_{p_s}: P_s times its later hits, in order
  u32 l = lam, used = 1u << (s & 31u);
  for (u32 s2 = 0; s2 < k; ++s2) {
    const u32 q2 = (u32)__shfl((int)qs, (int)s2), l2 = (u32)__shfl((int)lam, (int)s2);
    if (on && ((dh >> s2) & 1u)) {  // dh holds only pivots after s
      l = (l2 + l + 2u * ((u32)__popc(q2 & used) & 1u)) & 3u;
      used |= 1u << s2;
    }
  }
  const u32 e = (l - (pd & 3u)) & 3u;
  if (on) {
    bs->lam[s] = lam;
    bs->dsign[s] = e >> 1;
  }
  if (__ballot(on && (e & 1u)) && lane == 0) atomicOr(&st->flags, 1u);
}


// The hit masks and the pivot rows in one launch (they do not depend on each
// other): workgroups [0, mblocks) compute the masks, the others the rows.
__global__ __launch_bounds__(ROWS_T) void k_blk_masks_rows(const u64 *__restrict__ X, const u64 *__restrict__ Z,
                                                           const u64 *__restrict__ R, u64 *__restrict__ bm,
                                                           BlkState *__restrict__ bs,
                                                           u32 *__restrict__ patx, u32 *__restrict__ patz,
                                                           u32 *__restrict__ wpart, u32 *__restrict__ clist, u32 Ls,
                                                           u32 L, u32 K, u32 n, u32 mblocks) {
  if (blockIdx.x < mblocks)
    blk_masks(X, bm, bs, Ls, L, K, blockIdx.x);
  else
    blk_rows(X, Z, R, Ls, K, n, bs, patx, patz, wpart, clist, blockIdx.x - mblocks);
}

constexpr u32 BLK_PASS_T = 512;

// -------------------------------------------------------------- the pass
// Grid (row tiles of BLK_PASS_T words, column chunks). A thread owns one row
// word. The chunks split the block's list of supported columns (those where
// some pivot is not the identity, compacted by k_blk_masks_rows) evenly; a
// workgroup stages its share of the list in LDS (BLK_LIST entries at a
// time) and walks it with the row words of the next two columns loaded
// ahead. Per column (patterns uniform over the wave): XOR in the masks of
// the pivots with x (z) there, count |x & z| - |x' & z'| (mod 4) and the
// parities z_{P_s} . x_h. Columns are streamed with the non-temporal hint;
// unsupported columns are never touched.
constexpr u32 BLK_LIST = 2048;

__global__ __launch_bounds__(BLK_PASS_T) void k_blk_pass(u64 *__restrict__ X, u64 *__restrict__ Z,
                                                  const u64 *__restrict__ bm, const u32 *__restrict__ patx,
                                                  const u32 *__restrict__ patz, const BlkState *__restrict__ bs,
                                                  const u32 *__restrict__ clist, u64 *__restrict__ part, u32 Ls,
                                                  u32 L) {
  __shared__ u32 s_cols[BLK_LIST];
  const u32 k = bs->k;
  if (k == 0) return;  // the same for every workgroup
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 nc = bs->ncols;
  const u32 e0 = (u32)(((u64)blockIdx.y * nc) / gridDim.y), e1 = (u32)(((u64)(blockIdx.y + 1) * nc) / gridDim.y);
  u64 b[KB];
  u64 any = 0;
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {
    const u64 v = w < L ? bm[(size_t)s * Ls + w] : 0ULL;  // rows past k are allocated: load, then mask
    b[s] = s < k ? v : 0ULL;
    any |= b[s];
  }
  const bool act = any != 0;  // row words holding no hit row are left alone (and so are their partials)
  u64 yy = 0;          // z_{C_h} . x_h per row: XOR over columns of dz & x
  u64 d0 = 0, d1 = 0;  // |x & z| - |x' & z'| (mod 4), bit-sliced
  for (u32 c0 = e0; c0 < e1; c0 += BLK_LIST) {
    const u32 cn = min(e1 - c0, BLK_LIST);
    __syncthreads();  // the previous share of the list is consumed
    for (u32 i = threadIdx.x; i < cn; i += blockDim.x) s_cols[i] = clist[c0 + i];
    __syncthreads();
    if (!act) continue;
    // the row word of the next two columns is loaded ahead (the stores to
    // column j cannot alias them, which the compiler cannot see by itself)
    u64 xa = 0, za = 0, xb = 0, zb = 0;
    {
      const size_t oa = (size_t)s_cols[0] * Ls + w;
      xa = __builtin_nontemporal_load(X + oa);
      za = __builtin_nontemporal_load(Z + oa);
    }
    if (cn > 1) {
      const size_t ob = (size_t)s_cols[1] * Ls + w;
      xb = __builtin_nontemporal_load(X + ob);
      zb = __builtin_nontemporal_load(Z + ob);
    }
    for (u32 i = 0; i < cn; ++i) {
      const u32 j = s_cols[i];
      const size_t o = (size_t)j * Ls + w;
      const u64 x = xa, z = za;
      xa = xb;
      za = zb;
      if (i + 2 < cn) {
        const size_t o2 = (size_t)s_cols[i + 2] * Ls + w;
        xb = __builtin_nontemporal_load(X + o2);
        zb = __builtin_nontemporal_load(Z + o2);
      }
      const u32 px = patx[j], pz = patz[j];
      u64 dx = 0, dz = 0;
#pragma unroll
      for (u32 s = 0; s < KB; ++s) {  // all-ones / zero masks from the uniform patterns
        dx = xor_and(dx, b[s], 0u - ((px >> s) & 1u));
        dz = xor_and(dz, b[s], 0u - ((pz >> s) & 1u));
      }
      yy ^= dz & x;
      const u64 x2 = x ^ dx, z2 = z ^ dz;
      const u64 o1 = x & z, n1 = x2 & z2;
      const u64 plus = o1 & ~n1, minus = n1 & ~o1;
      d1 ^= d0 & plus;
      d0 ^= plus;
      d0 ^= minus;
      d1 ^= d0 & minus;
      if (px) __builtin_nontemporal_store(x2, X + o);
      if (pz) __builtin_nontemporal_store(z2, Z + o);
    }
  }
  if (!act) return;
  const size_t cs = (size_t)blockIdx.y * BLK_PART * Ls;
  part[cs + w] = d0;
  part[cs + Ls + w] = d1;
  part[cs + 2 * (size_t)Ls + w] = yy;
}

// -------------------------------------------------------------- chunk reduction
// A wave per (row word, field): lanes take every 64th chunk, then a butterfly
// combines them. Field 0 adds the 2-bit counters (mod 4), field 1 XORs the
// parity words. The result goes to chunk 0's slots. The grid has one column
// of workgroups more (of ROWS_T threads): its first does the block's pivot
// algebra (blk_algebra), the second nothing.
__global__ __launch_bounds__(ROWS_T) void k_blk_reduce(u64 *__restrict__ part, const u64 *__restrict__ bm,
                                                       const u32 *__restrict__ wpart, BlkState *__restrict__ bs,
                                                       MeasState *__restrict__ st, u32 Ls, u32 L, u32 nchunks,
                                                       u32 rblocks) {
  if (blockIdx.x == gridDim.x - 1) {  // uniform over the workgroup
    if (blockIdx.y == 0) blk_algebra(wpart, bs, st, rblocks);
    return;
  }
  const u32 k = bs->k;
  const u32 lane = threadIdx.x & 63u;
  const u32 w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const u32 f = blockIdx.y;
  if (w >= L) return;  // uniform over the wave
  u64 any = 0;
#pragma unroll
  for (u32 s = 0; s < KB; ++s)  // loads in flight together (rows past k: not used)
    any |= s < k ? bm[(size_t)s * Ls + w] : 0ULL;
  if (any == 0) return;  // k_blk_pass wrote nothing for this row word
  const size_t stride = (size_t)BLK_PART * Ls;
  if (f == 0) {
    u64 d0 = 0, d1 = 0;
#pragma unroll 4
    for (u32 c = lane; c < nchunks; c += 64u) {
      const u64 a0 = part[c * stride + w], a1 = part[c * stride + Ls + w];
      const u64 carry = d0 & a0;
      d0 ^= a0;
      d1 ^= a1 ^ carry;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const u64 o0 = shfl_xor_u64(d0, off), o1 = shfl_xor_u64(d1, off);
      const u64 carry = d0 & o0;
      d0 ^= o0;
      d1 ^= o1 ^ carry;
    }
    if (lane == 0) {
      part[w] = d0;
      part[Ls + w] = d1;
    }
  } else {
    const size_t o = 2 * (size_t)Ls + w;
    u64 y = 0;
#pragma unroll 4
    for (u32 c = lane; c < nchunks; c += 64u) y ^= part[c * stride + o];
    for (int off = 32; off > 0; off >>= 1) y ^= shfl_xor_u64(y, off);
    if (lane == 0) part[o] = y;
  }
}

// -------------------------------------------------------------- final
// Thread per row word (blocks of BLK_FIN_T): new signs of the hit rows from
// the lam algebra, then the special rows' signs (dsign, the coins). The hit
// masks stay in registers (the pivot conditions are uniform). The block's
// byte count (x and z of every supported column, read and written, for each
// row word holding a hit row) is added here too.
constexpr u32 BLK_FIN_T = 256;  // threads per workgroup of k_blk_signs_special

__device__ __forceinline__ void blk_signs(u64 *__restrict__ R, const u64 *__restrict__ bm,
                                          const u64 *__restrict__ part, const BlkState *__restrict__ bs,
                                          MeasState *__restrict__ st, MeasStats *__restrict__ stats, u32 Ls, u32 L,
                                          u32 K, u32 bid) {
  __shared__ u32 spv[KB], sfl[KB];  // per pivot: row, D-row sign (bit 0) and coin (bit 1)
  const u32 k = bs->k;
  if (k == 0) return;  // the same for every workgroup
  if (threadIdx.x < KB) {  // entries past k are not read
    spv[threadIdx.x] = bs->p[threadIdx.x];
    sfl[threadIdx.x] = (bs->dsign[threadIdx.x] ? 1u : 0u) | (bs->coin[threadIdx.x] ? 2u : 0u);
  }
  __syncthreads();
  const u32 w = bid * blockDim.x + threadIdx.x;
  const bool in = w < L;
  u64 b[KB];
#pragma unroll
  for (u32 s = 0; s < KB; ++s) b[s] = in ? bm[(size_t)s * Ls + w] : 0ULL;  // rows past k: not used
  u64 any = 0;
#pragma unroll
  for (u32 s = 0; s < KB; ++s)
    if (s < k) any |= b[s];
  const u32 nhit = (u32)__popcll(__ballot(any != 0));
  if ((threadIdx.x & 63u) == 0 && nhit) atomicAdd(&stats->block_bytes, (u64)nhit * 8ULL * 4ULL * bs->ncols);
  if (!in) return;
  u64 r = R[w];
  bool touched = false;
  if (any) {
    // chunk sums reduced by k_blk_reduce into chunk 0's slots
    const u64 d0 = part[w], d1 = part[Ls + w], yy = part[2 * (size_t)Ls + w];
    // lam = sum_s b_s lam(P_s) + 2 sum_{s<s'} b_s b_s' Qz[s'][s] + 2 r + 2 (z_{C_h} . x_h) + d
    u64 l0 = 0, l1 = 0;
#pragma unroll
    for (u32 s = 0; s < KB; ++s) {
      if (s < k) {
        const u32 lp = bs->lam[s], q = bs->Qz[s];
        if (lp & 1u) { l1 ^= l0 & b[s]; l0 ^= b[s]; }
        if (lp & 2u) l1 ^= b[s];
        u64 acc = 0;  // XOR of the earlier masks selected by row s of Qz
#pragma unroll
        for (u32 sp = 0; sp < s; ++sp)
          if ((q >> sp) & 1u) acc ^= b[sp];
        l1 ^= b[s] & acc;
      }
    }
    l1 ^= r ^ yy;
    {
      const u64 carry = l0 & d0;
      l0 ^= d0;
      l1 ^= d1 ^ carry;
    }
    if (l0 & any) atomicOr(&st->flags, 1u);
    r = (r & ~any) | (l1 & any);
    touched = true;
  }
  for (u32 s = 0; s < k; ++s) {
    const u32 p = spv[s];
    const u64 bit = 1ULL << (p & 63u);
    if (w == (p >> 6)) { r = (r & ~bit) | ((sfl[s] & 1u) ? bit : 0ULL); touched = true; }
    if (w == K + (p >> 6)) { r = (r & ~bit) | ((sfl[s] & 2u) ? bit : 0ULL); touched = true; }
  }
  if (touched) R[w] = r;
  if (w == 0) {
    stats->n_random += k;
    stats->blocks += 1;
  }
}

// Thread per column: the column's bits of the special rows, one
// read-modify-write per distinct row word holding pivots: D_{p_s} = P_s times
// its later hits, S_{p_s} = Z_{q_s}. The words are distinct, so a thread
// loads SPEC_B of them (x and z, both halves) before changing any: a memory
// round trip per SPEC_B words instead of one per word.
__device__ __forceinline__ void blk_special(u64 *__restrict__ X, u64 *__restrict__ Z, const u32 *__restrict__ patx,
                                            const u32 *__restrict__ patz, const BlkState *__restrict__ bs, u32 Ls,
                                            u32 K, u32 n, u32 bid) {
  __shared__ u32 spv[KB], sdh[KB], sqb[KB];  // per pivot: row, D-row factors, measured qubit
  const u32 k = bs->k;
  if (k == 0) return;  // the same for every workgroup
  const u32 tid = threadIdx.x;
  if (tid < KB) {  // entries past k are not read
    spv[tid] = bs->p[tid];
    sdh[tid] = bs->dhits[tid] | (1u << tid);
    sqb[tid] = bs->q[tid];
  }
  __syncthreads();
  const u32 j = bid * blockDim.x + tid;
  if (j >= n) return;
  const u32 px = patx[j], pz = patz[j];
  u64 *x = X + (size_t)j * Ls;
  u64 *z = Z + (size_t)j * Ls;
  const u32 nw = bs->nwords;
  for (u32 i0 = 0; i0 < nw; i0 += SPEC_B) {
    u64 dx[SPEC_B], dz[SPEC_B], sx[SPEC_B], sz[SPEC_B];
#pragma unroll
    for (u32 u = 0; u < SPEC_B; ++u) {
      if (i0 + u < nw) {  // uniform
        const u32 wd = bs->word[i0 + u];
        dx[u] = x[wd];
        dz[u] = z[wd];
        sx[u] = x[K + wd];
        sz[u] = z[K + wd];
      }
    }
#pragma unroll
    for (u32 u = 0; u < SPEC_B; ++u) {
      if (i0 + u < nw) {
        const u32 wd = bs->word[i0 + u], mem = bs->wmem[i0 + u];
        u64 mask = 0, xd = 0, zd = 0, zs = 0;
        for (u32 m = mem; m; m &= m - 1) {
          const u32 s = (u32)__builtin_ctz(m);
          const u64 bit = 1ULL << (spv[s] & 63u);
          const u32 dh = sdh[s];
          mask |= bit;
          if (__popc(px & dh) & 1) xd |= bit;
          if (__popc(pz & dh) & 1) zd |= bit;
          if (j == sqb[s]) zs |= bit;
        }
        x[wd] = (dx[u] & ~mask) | xd;
        z[wd] = (dz[u] & ~mask) | zd;
        x[K + wd] = sx[u] & ~mask;
        z[K + wd] = (sz[u] & ~mask) | zs;
      }
    }
  }
}


// -------------------------------------------------------------- symbolic signs (sampling sweep)
// With stabilizer signs kept as affine forms in the coins (sign column v =
// coefficient of coin v, column `count` = the constant), a block acts on the
// forms linearly. With every original sign set to 0 the block's algebra gives
// a constant c(h) per hit row (blk_signs writes it when run on a zeroed sign
// word array); the sign-dependent part is
//   r'(h) = r(h) ^ XOR_s b_s(h) Lin(P_s),  Lin(P_s) = r(S0_{p_s}) ^ XOR_{s' hits s} Lin(P_{s'}),
// and S_{p_s} becomes Z_{q_s} with its own coin (column m0 + s) as sign.

// Thread t <= m0 (m0 = the block's list position): sign column v = t
// (t < m0) or the constant (t = m0); bit s of svt[t] = coefficient of column
// v in Lin(P_s).
__device__ __forceinline__ void blk_sv_prep(const u64 *__restrict__ sg, u32 Ks, u32 count,
                                            const BlkState *__restrict__ bs, u32 *__restrict__ svt, u32 bid) {
  const u32 k = bs->k, m0 = bs->i0;
  const u32 t = bid * blockDim.x + threadIdx.x;
  if (k == 0 || t > m0) return;
  const u32 v = t < m0 ? t : count;
  const u32 nw = bs->nwords;
  u32 s0 = 0;  // coefficients of the original pivot rows
  for (u32 i0 = 0; i0 < nw; i0 += SPEC_B) {
    u64 wv[SPEC_B];
#pragma unroll
    for (u32 u = 0; u < SPEC_B; ++u) wv[u] = i0 + u < nw ? sg[(size_t)v * Ks + bs->word[i0 + u]] : 0ULL;
#pragma unroll
    for (u32 u = 0; u < SPEC_B; ++u) {
      if (i0 + u >= nw) break;
      for (u32 m = bs->wmem[i0 + u]; m; m &= m - 1) {
        const u32 s = (u32)__builtin_ctz(m);
        if ((wv[u] >> (bs->p[s] & 63u)) & 1ULL) s0 |= 1u << s;
      }
    }
  }
  u32 lin = 0;
  for (u32 s = 0; s < k; ++s) lin |= ((((s0 >> s) & 1u) ^ ((u32)__popc(lin & bs->hitS[s]) & 1u)) << s);
  svt[t] = lin;
}

// The sign update, the special rows and (sampling) the coefficients of the
// pivots' sign forms in one launch (none depends on another): workgroups
// [0, sblocks) take row words, [sblocks, sblocks + cblocks) columns, the
// rest the sign-form columns (sg != nullptr only on the sampling path).
__global__ __launch_bounds__(BLK_FIN_T) void k_blk_signs_special(
    u64 *__restrict__ R, const u64 *__restrict__ bm, const u64 *__restrict__ part, const BlkState *__restrict__ bs,
    MeasState *__restrict__ st, MeasStats *__restrict__ stats, u64 *__restrict__ X, u64 *__restrict__ Z,
    const u32 *__restrict__ patx, const u32 *__restrict__ patz, const u64 *__restrict__ sg, u32 Ks, u32 count,
    u32 *__restrict__ svt, u32 Ls, u32 L, u32 K, u32 n, u32 sblocks, u32 cblocks) {
  if (blockIdx.x < sblocks)
    blk_signs(R, bm, part, bs, st, stats, Ls, L, K, blockIdx.x);
  else if (blockIdx.x < sblocks + cblocks)
    blk_special(X, Z, patx, patz, bs, Ls, K, n, blockIdx.x - sblocks);
  else
    blk_sv_prep(sg, Ks, count, bs, svt, blockIdx.x - sblocks - cblocks);
}

// Grid (stabilizer-word tiles, workgroups over column chunks of SV_CHUNK):
// thread per stabilizer word; workgroup y takes the chunks y, y + gridDim.y,
// ... of the columns t in [0, m0 + k]: t < m0 coin columns, m0 <= t < m0 + k
// this block's coins, t = m0 + k the constant. Up to SV_MAX_Y workgroups
// along y, so that late in a sweep (thousands of coin columns) a workgroup
// walks a few chunks, not dozens, one memory round trip each.
constexpr u32 SV_CHUNK = 16, SV_GROUP = 16, SV_MAX_Y = 512;

__global__ __launch_bounds__(64) void k_blk_sv_update(u64 *__restrict__ sg, u32 Ks, u32 count,
                                                       const BlkState *__restrict__ bs, const u64 *__restrict__ bm,
                                                       const u32 *__restrict__ svt, const u64 *__restrict__ cvec,
                                                       u32 Ls, u32 K) {
  const u32 k = bs->k, m0 = bs->i0;
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;  // stabilizer row word
  if (k == 0 || w >= K || blockIdx.y * SV_CHUNK > m0 + k) return;
  u64 b[KB];
#pragma unroll
  for (u32 s = 0; s < KB; ++s) {  // rows past k are allocated: load, then mask
    const u64 v = bm[(size_t)s * Ls + K + w];
    b[s] = s < k ? v : 0ULL;
  }
  u64 smask = 0;  // rows S_{p_s} in this word
  for (u32 s = 0; s < k; ++s)
    if ((bs->p[s] >> 6) == w) smask |= 1ULL << (bs->p[s] & 63u);
  for (u32 tlo = blockIdx.y * SV_CHUNK; tlo <= m0 + k; tlo += gridDim.y * SV_CHUNK) {
    const u32 thi = min(tlo + SV_CHUNK, m0 + k + 1);
    // columns in groups of SV_GROUP: the group's loads are in flight together
    for (u32 t0 = tlo; t0 < thi; t0 += SV_GROUP) {
      u64 val[SV_GROUP];
#pragma unroll
      for (u32 i = 0; i < SV_GROUP; ++i) {
        const u32 t = t0 + i;
        const u32 v = t < m0 + k ? t : count;
        val[i] = t < thi ? sg[(size_t)v * Ks + w] : 0ULL;
      }
#pragma unroll
      for (u32 i = 0; i < SV_GROUP; ++i) {
        const u32 t = t0 + i;
        if (t >= thi) continue;
        const bool own = t >= m0 && t < m0 + k;  // a coin of this block
        const u32 v = t < m0 + k ? t : count;
        u64 x = val[i];
        if (!own) {
          const u32 lin = svt[t < m0 ? t : m0];
          u64 acc = 0;
#pragma unroll
          for (u32 s = 0; s < KB; ++s) acc = xor_and(acc, b[s], 0u - ((lin >> s) & 1u));
          x ^= acc;
          if (v == count) x ^= cvec[K + w];
        }
        if (smask) {
          u64 set = 0;
          if (own) {
            const u32 p = bs->p[t - m0];
            if ((p >> 6) == w) set = 1ULL << (p & 63u);
          }
          x = (x & ~smask) | set;
        }
        sg[(size_t)v * Ks + w] = x;
      }
    }
  }
}

// -------------------------------------------------------------- launchers
// Stage 0: the sequential pivot step on the cursor's next measurements (it
// writes BlkState::k, which every later kernel of the block reads, and
// advances the cursor).
hipError_t launch_blk_pivots(const TabDev &t, Cursor *cur, const BlkBuffers &b, u32 waves, u64 *zero_words,
                             u32 nzero, hipStream_t s) {
  const u32 tiles = std::max<u32>(1, cdiv(t.K, 64));
  if (waves == PIVOT_AUTO && tiles <= PR_WAVES)
    hipLaunchKernelGGL(k_blk_pivots_reg, dim3(1), dim3(64 * tiles), 0, s, t.X, t.Ls, t.K, cur, b.bs, zero_words,
                       nzero);
  else {
    const u32 G = cdiv(t.K, 256);  // chunks of the first-nonzero search (fz in wpart: KB * G <= 4 KB K words)
    hipLaunchKernelGGL(k_blk_firstnz, dim3(G, KB), dim3(256), 0, s, t.X, t.Ls, t.K, cur, b.wpart, G);
    hipLaunchKernelGGL(k_blk_pivots, dim3(1), dim3(64 * std::min<u32>({PW_WAVES, tiles, waves})), 0, s, t.X,
                       t.Ls, t.K, cur, b.bs, zero_words, nzero, b.wpart, G);
  }
  return hipGetLastError();
}

// Stage 1: hit masks, pivot rows and their algebra.
hipError_t launch_blk_prep(const TabDev &t, const BlkBuffers &b, hipStream_t s) {
  const u32 mblocks = cdiv(t.L, ROWS_T), rblocks = cdiv(t.n, ROWS_T);
  hipLaunchKernelGGL(k_blk_masks_rows, dim3(mblocks + rblocks), dim3(ROWS_T), 0, s, t.X, t.Z, t.R, b.bm, b.bs,
                     b.patx, b.patz, b.wpart, b.clist, t.Ls, t.L, t.K, t.n, mblocks);
  return hipGetLastError();
}

// Stage 2: the streaming pass over the tableau.
hipError_t launch_blk_pass(const TabDev &t, const BlkBuffers &b, u32 cpc, hipStream_t s) {
  const u32 nchunks = cdiv(t.n, cpc);
  hipLaunchKernelGGL(k_blk_pass, dim3(cdiv(t.L, BLK_PASS_T), nchunks), dim3(BLK_PASS_T), 0, s, t.X, t.Z, b.bm, b.patx,
                     b.patz, b.bs, b.clist, b.part, t.Ls, t.L);
  return hipGetLastError();
}

// Stage 3: chunk reduction with the pivot algebra, then signs, the special
// rows and (sampling: sg != nullptr) the pivots' sign-form coefficients svt.
hipError_t launch_blk_final(const TabDev &t, const BlkBuffers &b, MeasState *st, MeasStats *stats, u32 cpc,
                            const u64 *sg, u32 Ks, u32 count, u32 *svt, hipStream_t s) {
  const u32 nchunks = cdiv(t.n, cpc);
  // k_blk_reduce: a wave per (row word, field), then one workgroup for the pivot algebra
  hipLaunchKernelGGL(k_blk_reduce, dim3(cdiv(t.L, ROWS_T / 64) + 1, 2), dim3(ROWS_T), 0, s, b.part, b.bm, b.wpart,
                     b.bs, st, t.Ls, t.L, nchunks, cdiv(t.n, ROWS_T));
  const u32 sblocks = cdiv(t.L, BLK_FIN_T), cblocks = cdiv(t.n, BLK_FIN_T);
  const u32 vblocks = sg ? cdiv(count + 1, BLK_FIN_T) : 0u;  // sign-form columns 0 .. count
  hipLaunchKernelGGL(k_blk_signs_special, dim3(sblocks + cblocks + vblocks), dim3(BLK_FIN_T), 0, s, t.R, b.bm,
                     b.part, b.bs, st, stats, t.X, t.Z, b.patx, b.patz, sg, Ks, count, svt, t.Ls, t.L, t.K, t.n,
                     sblocks, cblocks);
  return hipGetLastError();
}

// Symbolic signs after a block whose pass, special rows and svt are done;
// cvec holds the constants c(h) (the block ran with it as its zeroed sign
// array).
// The block's list position is read on the device, so the grid covers every
// position up to `count`.
hipError_t launch_blk_sv(u64 *sg, u32 Ks, u32 count, const BlkBuffers &b, const u32 *svt, const u64 *cvec, u32 Ls,
                         u32 K, hipStream_t s) {
  const u32 ychunks = std::min<u32>(SV_MAX_Y, cdiv(count + 1, SV_CHUNK));
  hipLaunchKernelGGL(k_blk_sv_update, dim3(cdiv(K, 64), ychunks), dim3(64), 0, s, sg, Ks, count, b.bs, b.bm, svt,
                     cvec, Ls, K);
  return hipGetLastError();
}

}  // namespace sq
