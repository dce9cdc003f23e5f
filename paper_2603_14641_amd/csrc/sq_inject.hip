// Z measurement on the operator tableau by CX injection (the paper's
// collapse, Algorithm alg:stim), two launches per measured qubit:
//   k_inj_pivot  pivot p (smallest stabilizer position with x_q(S_p) = 1),
//                the target mask T = {t > p : x_q(S_t) = 1} snapshotted and
//                its nonzero words compacted in order (the role of Algorithm
//                alg:compactPivots), and the decisions that only column q
//                fixes; deterministic outcomes are just B_q's sign;
//   k_inj_apply  every column j at once: the CX injections from p into every
//                target, the pivot rotation (Algorithm alg:assembly: H, or
//                the inverse-phase rotation when x_q(D_p) = 1 after the
//                injections) and the X injection when the sign differs from
//                the coin.
//
// In the column-major layout the injections are independent per column.
// At column j the injection into target t (in increasing t) does, with
// c = x_j(S_p), d_t = x_j(D_t), s_t = x_j(S_t) and P_t = x_j(D_p) as the
// earlier targets left it:
//   sign_B(j) ^= c & d_t & ~(P_t ^ s_t);  s_t ^= c;  P_{t+1} = P_t ^ d_t
// (and the same on the z bits for the sign of A_j), so P_t is the initial
// x_j(D_p) XOR an exclusive prefix XOR of the d bits over the targets: the
// loop-carried dependency the paper unfolds into a prefix-XOR (equations
// CXSign and zc). Here it is a scan along the column: an in-word shift-XOR
// scan of the target bits, a wave ballot over the words a wave holds, and a
// carry across the wave's rounds. Everything a column needs is in the column
// itself plus the pivot's bits, so the pass reads each column's target words
// once and writes back only the stabilizer words where S_p has a 1.
#include "sq_device.h"

namespace sq {

// Bit b: XOR of the bits of v below b.
__device__ __forceinline__ u64 prefix_xor_excl(u64 v) {
  u64 y = v;
  y ^= y << 1;
  y ^= y << 2;
  y ^= y << 4;
  y ^= y << 8;
  y ^= y << 16;
  y ^= y << 32;
  return y ^ v;
}

// One workgroup of 1024 threads (16 waves). Reads the cursor like k_pivot
// (one measurement per slot), finds p in the stabilizer half of X column q,
// and for a random outcome snapshots T into mask[0..K), writes the indices
// of its nonzero words in increasing order to tw[0..nT), and evaluates
// column q's own injections: x_q(D_p) after them (which rotation follows)
// and the sign of B_q after them (whether the X injection follows, so that
// the sign, which is the outcome, equals the coin). At column q every target
// has s_t = c = 1, so its sign term is d_t & P_t.
__global__ __launch_bounds__(1024) void k_inj_pivot(const u64 *__restrict__ X, const u64 *__restrict__ R, u32 Ls,
                                                    u32 K, Cursor *__restrict__ cur, MeasState *__restrict__ st,
                                                    u64 *__restrict__ mask, u32 *__restrict__ tw,
                                                    MeasStats *__restrict__ stats) {
  __shared__ u32 s_min, s_act, s_q, s_i;
  __shared__ u32 s_cnt[16], s_par[16], s_g[16];
  const u32 tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nwaves = blockDim.x >> 6;
  if (tid == 0) {
    s_min = 0xFFFFFFFFu;
    const u32 i = cur->i;
    const u32 act = i < cur->end ? 1u : 0u;
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
  for (u32 w = tid; w < K; w += blockDim.x)
    if (col[K + w] != 0) { first = w; break; }
  for (int off = 32; off > 0; off >>= 1) first = min(first, (u32)__shfl_xor((int)first, off));
  if (lane == 0 && first != 0xFFFFFFFFu) atomicMin(&s_min, first);
  __syncthreads();
  const u32 wmin = s_min;
  const u32 sign_b = (u32)(R[K + (q >> 6)] >> (q & 63u)) & 1u;
  if (wmin == 0xFFFFFFFFu) {  // deterministic: the outcome is B_q's sign
    if (tid == 0) {
      st->p = -1;
      st->q = q;
      st->i = i;
      if (cur->out_bits) cur->out_bits[i] = (uint8_t)sign_b;
      if (cur->out_rand) cur->out_rand[i] = 0;
      cur->i = i + 1;
      stats->n_det += 1;
    }
    return;
  }
  const u32 p = wmin * 64u + (u32)__builtin_ctzll(col[K + wmin]);
  const u32 wp = p >> 6;
  const u64 above = (~0ULL << (p & 63u)) << 1;  // bits > p of word wp (0 when p & 63 == 63)
  u32 base = 0;                                   // compacted words so far
  u32 carry = (u32)(col[wp] >> (p & 63u)) & 1u;  // x_q(D_p), then XOR of the d bits so far
  u32 g = 0;                                      // this thread's sign terms
  for (u32 w0 = wp; w0 < K; w0 += blockDim.x) {
    const u32 w = w0 + tid;
    u64 m = 0, d = 0;
    if (w < K) {
      m = col[K + w];
      if (w == wp) m &= above;
      mask[w] = m;
      d = col[w] & m;
    }
    const u64 bal = __ballot(m != 0);
    const u32 par = (u32)__popcll(d) & 1u;
    const u64 pb = __ballot(par);
    if (lane == 0) {
      s_cnt[wave] = (u32)__popcll(bal);
      s_par[wave] = (u32)__popcll(pb) & 1u;
    }
    __syncthreads();
    u32 wbase = 0, wpar = 0, tcnt = 0, tpar = 0;
    for (u32 v = 0; v < nwaves; ++v) {
      if (v < wave) {
        wbase += s_cnt[v];
        wpar ^= s_par[v];
      }
      tcnt += s_cnt[v];
      tpar ^= s_par[v];
    }
    if (m != 0) tw[base + wbase + (u32)__popcll(bal & lanemask_lt())] = w;
    const u32 pre = carry ^ wpar ^ ((u32)__popcll(pb & lanemask_lt()) & 1u);
    const u64 P = prefix_xor_excl(d) ^ (pre ? ~0ULL : 0ULL);
    g ^= (u32)__popcll(d & P) & 1u;
    base += tcnt;
    carry ^= tpar;
    __syncthreads();
  }
  const u64 gb = __ballot(g);
  if (lane == 0) s_g[wave] = (u32)__popcll(gb) & 1u;
  __syncthreads();
  if (tid == 0) {
    u32 G = 0;
    for (u32 v = 0; v < nwaves; ++v) G ^= s_g[v];
    const u32 c = coin_bit(cur->seed, cur->shot, cur->meas_base + i);
    const u32 invp = carry;           // x_q(D_p) after the injections
    const u32 flip = sign_b ^ G ^ c;  // the sign after injections and rotation differs from the coin
    st->p = (int32_t)p;
    st->q = q;
    st->i = i;
    st->ncols = base;
    st->coin = c;
    st->inj = invp | (flip << 1);
    if (cur->out_bits) cur->out_bits[i] = (uint8_t)c;
    if (cur->out_rand) cur->out_rand[i] = 1;
    cur->i = i + 1;
    stats->n_random += 1;
  }
}

// A wave per column j (all n columns, q included). Loads the pivot's four
// bits at j, walks the compacted target words (lane l takes entries l,
// l + 64, ...), flips the stabilizer words where S_p has a 1 and scans the
// destabilizer bits, then applies the rotation and the X injection to the
// pivot pair and the column's two signs. The pair's words may have been
// rewritten by the scan, so the pair's bit changes go to pair[j] (bit 0:
// x of S_p, 1: x of D_p, 2: z of S_p, 3: z of D_p) and k_inj_pair applies
// them after this kernel; signs of 64 columns share a word (atomic XORs).
// Byte accounting: per column, read the two destabilizer words of each
// target word, and read and write the stabilizer word of X (Z) where the
// pivot has x (z).
__global__ __launch_bounds__(256) void k_inj_apply(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ R,
                                                   u32 Ls, u32 K, u32 n, const MeasState *__restrict__ st,
                                                   const u64 *__restrict__ mask, const u32 *__restrict__ tw,
                                                   uint8_t *__restrict__ pair, MeasStats *__restrict__ stats) {
  const int32_t ps = st->p;
  if (ps < 0) return;
  __shared__ u32 s_cnt;
  const u32 lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const u32 j = blockIdx.x * wpb + wave;
  const u32 p = (u32)ps, wp = p >> 6, sh = p & 63u;
  const u32 nT = st->ncols, inj = st->inj;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  if (j < n) {
    u64 *xc = X + (size_t)j * Ls;
    u64 *zc = Z + (size_t)j * Ls;
    const u32 cx = (u32)(xc[K + wp] >> sh) & 1u, cz = (u32)(zc[K + wp] >> sh) & 1u;
    const u32 d0x = (u32)(xc[wp] >> sh) & 1u, d0z = (u32)(zc[wp] >> sh) & 1u;
    u32 carx = d0x, carz = d0z, gx = 0, gz = 0;
    // dense target list (every word from wp on holds a target, the usual
    // case): the word index is the list index, so no list load
    const bool dense = nT == K - wp;
#pragma unroll 2
    for (u32 b = 0; b < nT; b += 64) {
      const u32 e = b + lane;
      u64 xd = 0, zd = 0, xs = 0, zs = 0;
      if (e < nT) {
        const u32 w = dense ? wp + e : tw[e];
        const u64 m = mask[w];
        xd = __builtin_nontemporal_load(xc + w) & m;
        zd = __builtin_nontemporal_load(zc + w) & m;
        if (cx) {
          xs = __builtin_nontemporal_load(xc + K + w);
          __builtin_nontemporal_store(xs ^ m, xc + K + w);
        }
        if (cz) {
          zs = __builtin_nontemporal_load(zc + K + w);
          __builtin_nontemporal_store(zs ^ m, zc + K + w);
        }
      }
      const u64 bx = __ballot((u32)__popcll(xd) & 1u), bz = __ballot((u32)__popcll(zd) & 1u);
      if (cx) {
        const u32 pre = carx ^ ((u32)__popcll(bx & lanemask_lt()) & 1u);
        const u64 P = prefix_xor_excl(xd) ^ (pre ? ~0ULL : 0ULL);
        gx ^= (u32)__popcll(xd & ~(P ^ xs)) & 1u;
      }
      if (cz) {
        const u32 pre = carz ^ ((u32)__popcll(bz & lanemask_lt()) & 1u);
        const u64 P = prefix_xor_excl(zd) ^ (pre ? ~0ULL : 0ULL);
        gz ^= (u32)__popcll(zd & ~(P ^ zs)) & 1u;
      }
      carx ^= (u32)__popcll(bx) & 1u;
      carz ^= (u32)__popcll(bz) & 1u;
    }
    u32 sb = (u32)__popcll(__ballot(gx)) & 1u;  // change of the sign of B_j
    u32 sa = (u32)__popcll(__ballot(gz)) & 1u;  // change of the sign of A_j
    u32 sx = cx, dx = carx, sz = cz, dz = carz;
    if (inj & 1u) {  // inverse-phase rotation (x_q(D_p) = 1)
      sb ^= sx & (dx ^ 1u);
      sx ^= dx;
      sa ^= sz & (dz ^ 1u);
      sz ^= dz;
    } else {  // Hadamard
      sb ^= sx & dx;
      { const u32 v = sx; sx = dx; dx = v; }
      sa ^= sz & dz;
      { const u32 v = sz; sz = dz; dz = v; }
    }
    if (inj & 2u) {  // X injection
      sb ^= dx;
      sa ^= dz;
    }
    if (lane == 0) {
      pair[j] = (uint8_t)((sx ^ cx) | ((dx ^ d0x) << 1) | ((sz ^ cz) << 2) | ((dz ^ d0z) << 3));
      if (sb) atomicXor(R + K + (j >> 6), 1ULL << (j & 63u));
      if (sa) atomicXor(R + (j >> 6), 1ULL << (j & 63u));
      atomicAdd(&s_cnt, cx + cz);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const u32 j0 = blockIdx.x * wpb;
    const u32 cols = j0 < n ? min(wpb, n - j0) : 0u;
    atomicAdd(&stats->inject_bytes, (unsigned long long)8ull * nT * (2ull * cols + 2ull * s_cnt));
  }
}

// Thread per column: the pivot pair's bit changes recorded by k_inj_apply.
__global__ void k_inj_pair(u64 *__restrict__ X, u64 *__restrict__ Z, u32 Ls, u32 K, u32 n,
                           const MeasState *__restrict__ st, const uint8_t *__restrict__ pair) {
  const int32_t ps = st->p;
  if (ps < 0) return;
  const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const u32 c = pair[j];
  if (!c) return;
  const u32 wp = (u32)ps >> 6;
  const u64 bit = 1ULL << ((u32)ps & 63u);
  u64 *xc = X + (size_t)j * Ls, *zc = Z + (size_t)j * Ls;
  if (c & 1u) xc[K + wp] ^= bit;
  if (c & 2u) xc[wp] ^= bit;
  if (c & 4u) zc[K + wp] ^= bit;
  if (c & 8u) zc[wp] ^= bit;
}

hipError_t launch_inj_pivot(const TabDev &t, Cursor *cur, MeasState *st, u64 *mask, u32 *tw, MeasStats *stats,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_inj_pivot, dim3(1), dim3(1024), 0, s, t.X, t.R, t.Ls, t.K, cur, st, mask, tw, stats);
  return hipGetLastError();
}

hipError_t launch_inj_apply(const TabDev &t, const MeasState *st, const u64 *mask, const u32 *tw, uint8_t *pair,
                            MeasStats *stats, hipStream_t s) {
  hipLaunchKernelGGL(k_inj_apply, dim3(cdiv(t.n, 4)), dim3(256), 0, s, t.X, t.Z, t.R, t.Ls, t.K, t.n, st, mask, tw,
                     pair, stats);
  hipLaunchKernelGGL(k_inj_pair, dim3(cdiv(t.n, 256)), dim3(256), 0, s, t.X, t.Z, t.Ls, t.K, t.n, st, pair);
  return hipGetLastError();
}

}  // namespace sq
