// Batched circuits: one persistent launch runs many independent circuits,
// one workgroup per circuit at a time. A workgroup takes the next circuit
// from an atomic counter (circuits are ordered largest first), prepares
// |0...0>, applies all its gate passes, runs the symbolic-sign measurement
// sweep of its measured list and evaluates every requested shot. The
// arithmetic is exactly that of the single-tableau path (sq_gates.hip,
// sq_measure.hip, sq_sample.hip); only the work distribution differs:
//   * thread (word lane w0, slice s) owns row words w = w0 + k*Lw; under
//     gates rows are independent, so a thread walks every group of its slice
//     over its words and passes are separated by one workgroup barrier;
//   * in the rowsum, slice s handles the pivot columns j = s (mod S) of its
//     words; the 2-bit phase counters of the slices are added in LDS;
//   * destabilizer signs are never needed for outcomes and are not kept.
#include "sq_device.h"

namespace sq {

constexpr u32 BW = 2;  // row words per thread in the batched kernel (L <= BW * blockDim)
constexpr u32 GB = 4;  // gate groups loaded together per thread

__device__ __forceinline__ void bapply(u64 ops, u64 &xa, u64 &za, u64 &xb, u64 &zb, u64 &s) {
  for (; ops != 0; ops >>= 4) {
    switch ((u32)(ops & 15ULL)) {
      case UOP_H_A: { s ^= xa & za; const u64 t = xa; xa = za; za = t; } break;
      case UOP_S_A: s ^= xa & za; za ^= xa; break;
      case UOP_SDG_A: s ^= xa & ~za; za ^= xa; break;
      case UOP_X_A: s ^= za; break;
      case UOP_Y_A: s ^= xa ^ za; break;
      case UOP_Z_A: s ^= xa; break;
      case UOP_H_B: { s ^= xb & zb; const u64 t = xb; xb = zb; zb = t; } break;
      case UOP_S_B: s ^= xb & zb; zb ^= xb; break;
      case UOP_SDG_B: s ^= xb & ~zb; zb ^= xb; break;
      case UOP_X_B: s ^= zb; break;
      case UOP_Y_B: s ^= xb ^ zb; break;
      case UOP_Z_B: s ^= xb; break;
      case UOP_CX_AB: s ^= xa & zb & ~(xb ^ za); xb ^= xa; za ^= zb; break;
      case UOP_CX_BA: s ^= xb & za & ~(xa ^ zb); xa ^= xb; zb ^= za; break;
      case UOP_CZ: { s ^= xa & xb & (za ^ zb); const u64 ta = za ^ xb; zb ^= xa; za = ta; } break;
      default: break;
    }
  }
}

// Limits of the batched path: L = 2 ceil(n/64) <= BATCH_MAX_WORDS (n <= 16384),
// at most 512 threads (L <= BW * blockDim), measured lists shorter than
// 64 * BATCH_MAX_WORDS; the LDS arrays below are sized for them (32 KB).
constexpr u32 BATCH_MAX_WORDS = 512;
constexpr u32 BATCH_MAX_BLOCK = 512;

__global__ __launch_bounds__(512) void k_batch(const BatchItem *__restrict__ items, u32 nitems,
                                               u32 *__restrict__ next) {
  __shared__ u32 s_item, s_min, s_flags;
  __shared__ int s_acc[BATCH_MAX_BLOCK / 64];
  __shared__ u64 s_px[BATCH_MAX_WORDS / 2], s_pz[BATCH_MAX_WORDS / 2];  // pivot row (n bits), or the A mask
  __shared__ u64 s_sgn[BATCH_MAX_WORDS];        // gate signs, then S_p's sign bitmap
  __shared__ u64 s_m[BATCH_MAX_WORDS];          // rowsum mask (column q before the pass)
  __shared__ u64 s_c0[BW * BATCH_MAX_BLOCK], s_c1[BW * BATCH_MAX_BLOCK];  // per-slice phase counters
  const u32 tid = threadIdx.x, T = blockDim.x, lane = tid & 63u, wave = tid >> 6, nwaves = T >> 6;

  for (;;) {
    if (tid == 0) s_item = atomicAdd(next, 1u);
    __syncthreads();
    const u32 it = s_item;
    __syncthreads();
    if (it >= nitems) return;
    const BatchItem d = items[it];
    const u32 n = d.n, K = (n + 63) / 64, L = 2 * K, Ls = d.Ls, Ks = d.Ks, CW = d.CW, count = d.count;
    u64 *X = d.X, *Z = d.Z, *sg = d.sg;
    u64 *sgc = sg + (size_t)count * Ks;
    // thread geometry: word lanes and slices
    const u32 Lw = min(L, T);
    const u32 S = T / Lw;
    const u32 w0 = tid % Lw, sl = tid / Lw;
    const bool active = sl < S;
    const u32 nw = (L + Lw - 1) / Lw;  // words per thread (<= BW)

    // ---- |0...0>: zero X, Z and the sign columns; D_i = X_i, S_i = Z_i
    for (size_t k = tid; k < (size_t)n * Ls; k += T) { X[k] = 0; Z[k] = 0; }
    for (size_t k = tid; k < (size_t)(count + 1) * Ks; k += T) sg[k] = 0;
    for (u32 k = tid; k < L; k += T) s_sgn[k] = 0;
    if (tid == 0) s_flags = 0;
    __syncthreads();
    for (u32 i = tid; i < n; i += T) {
      X[(size_t)i * Ls + (i >> 6)] = 1ULL << (i & 63u);
      Z[(size_t)i * Ls + K + (i >> 6)] = 1ULL << (i & 63u);
    }
    __syncthreads();

    // ---- gate passes
    u64 sgn[BW] = {0, 0};
    for (u32 p = 0; p < d.npasses; ++p) {
      const u32 g0 = d.pass_off[p], g1 = d.pass_off[p + 1];
      if (active) {
        // GB groups of this slice at a time: all loads first, then apply and store
        // (groups of one pass touch disjoint columns)
        for (u32 gs = g0 + sl; gs < g1; gs += S * GB) {
          Group G[GB];
          u32 nb = 0;
#pragma unroll
          for (u32 b = 0; b < GB; ++b)
            if (gs + b * S < g1) { G[b] = d.groups[gs + b * S]; nb = b + 1; }
          for (u32 k = 0; k < nw; ++k) {
            const u32 w = w0 + k * Lw;
            if (w >= L) break;
            u64 xa[GB], za[GB], xb[GB], zb[GB];
#pragma unroll
            for (u32 b = 0; b < GB; ++b) {
              xa[b] = za[b] = xb[b] = zb[b] = 0;
              if (b < nb) {
                const size_t ca = (size_t)(G[b].q0 & GQ_MASK) * Ls + w;
                xa[b] = X[ca];
                za[b] = Z[ca];
                if (G[b].q1 != G_SINGLE) {
                  const size_t cb = (size_t)G[b].q1 * Ls + w;
                  xb[b] = X[cb];
                  zb[b] = Z[cb];
                }
              }
            }
#pragma unroll
            for (u32 b = 0; b < GB; ++b) {
              if (b >= nb) break;
              bapply(G[b].ops, xa[b], za[b], xb[b], zb[b], sgn[k]);
              const size_t ca = (size_t)(G[b].q0 & GQ_MASK) * Ls + w;
              if (G[b].q0 & GD_XA) X[ca] = xa[b];
              if (G[b].q0 & GD_ZA) Z[ca] = za[b];
              if (G[b].q1 != G_SINGLE) {
                const size_t cb = (size_t)G[b].q1 * Ls + w;
                if (G[b].q0 & GD_XB) X[cb] = xb[b];
                if (G[b].q0 & GD_ZB) Z[cb] = zb[b];
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (active)
      for (u32 k = 0; k < nw; ++k) {
        const u32 w = w0 + k * Lw;
        if (w < L && sgn[k]) atomicXor(&s_sgn[w], sgn[k]);
      }
    __syncthreads();
    for (u32 w = tid; w < K; w += T) sgc[w] = s_sgn[K + w];  // stabilizer signs -> constant column
    __syncthreads();

    // ---- symbolic measurement sweep
    for (u32 i = 0; i < count; ++i) {
      const u32 q = d.qubits[i];
      const u64 *colq = X + (size_t)q * Ls;
      if (tid == 0) s_min = 0xFFFFFFFFu;
      __syncthreads();
      u32 first = 0xFFFFFFFFu;
      for (u32 w = tid; w < K; w += T)
        if (colq[K + w] != 0) { first = w; break; }
      for (int off = 32; off > 0; off >>= 1) first = min(first, (u32)__shfl_xor((int)first, off));
      if (lane == 0 && first != 0xFFFFFFFFu) atomicMin(&s_min, first);
      __syncthreads();
      const u32 wmin = s_min;
      if (wmin != 0xFFFFFFFFu) {
        // ------------------------------------------------ random case
        const u32 p = wmin * 64u + (u32)__builtin_ctzll(colq[K + wmin]);
        const u32 wd = p >> 6, ws = K + wd;
        const u64 bit = 1ULL << (p & 63u);
        // (1) pivot row and S_p's sign bitmap (bit v: coin v for v < i, bit i:
        // the constant) into LDS; masks = column q before the pass rewrites it
        for (u32 jb = 0; jb < n; jb += T) {
          const u32 j = jb + tid;
          const u32 xb = (j < n) ? (u32)(X[(size_t)j * Ls + ws] >> (p & 63u)) & 1u : 0u;
          const u32 zb = (j < n) ? (u32)(Z[(size_t)j * Ls + ws] >> (p & 63u)) & 1u : 0u;
          const u64 bx = __ballot(xb), bz = __ballot(zb);
          if (lane == 0 && j < n) { s_px[j >> 6] = bx; s_pz[j >> 6] = bz; }
        }
        for (u32 vb = 0; vb <= i; vb += T) {
          const u32 v = vb + tid;
          u32 b = 0;
          if (v <= i) {
            const u32 col = (v == i) ? count : v;
            b = (u32)(sg[(size_t)col * Ks + wd] >> (p & 63u)) & 1u;
          }
          const u64 bb = __ballot(b);
          if (lane == 0 && v <= i) s_sgn[v >> 6] = bb;
        }
        for (u32 w = tid; w < L; w += T) {
          u64 v = colq[w];
          if (w == wd || w == ws) v &= ~bit;
          s_m[w] = v;
        }
        __syncthreads();
        // (2) rowsum: slice sl takes pivot columns j = sl (mod S) of its words
        if (active) {
          u64 m[BW] = {0, 0}, a0[BW] = {0, 0}, a1[BW] = {0, 0};
          for (u32 k = 0; k < nw; ++k) {
            const u32 w = w0 + k * Lw;
            if (w < L) m[k] = s_m[w];
          }
          for (u32 j = sl; j < n; j += S) {
            const u32 px = (u32)(s_px[j >> 6] >> (j & 63u)) & 1u, pz = (u32)(s_pz[j >> 6] >> (j & 63u)) & 1u;
            if (!(px | pz)) continue;
            const size_t cj = (size_t)j * Ls;
            for (u32 k = 0; k < nw; ++k) {
              if (!m[k]) continue;
              const u32 w = w0 + k * Lw;
              const u64 x = X[cj + w], z = Z[cj + w];
              u64 plus, minus;
              if (px && !pz) { plus = x & z; minus = ~x & z; }
              else if (px) { plus = ~x & z; minus = x & ~z; }
              else { plus = x & ~z; minus = x & z; }
              plus &= m[k];
              minus &= m[k];
              a1[k] ^= a0[k] & plus;
              a0[k] ^= plus;
              a0[k] ^= minus;
              a1[k] ^= a0[k] & minus;
              if (px) X[cj + w] = x ^ m[k];
              if (pz) Z[cj + w] = z ^ m[k];
            }
          }
          // masked stabilizer rows take S_p's sign vector (slice 0 does it)
          if (sl == 0)
            for (u32 k = 0; k < nw; ++k) {
              const u32 w = w0 + k * Lw;
              if (w < K || w >= L || !m[k]) continue;
              for (u32 vw = 0; vw <= (i >> 6); ++vw) {
                u64 bits = s_sgn[vw];
                while (bits) {
                  const u32 v = vw * 64u + (u32)__builtin_ctzll(bits);
                  bits &= bits - 1;
                  const u32 col = (v == i) ? count : v;
                  sg[(size_t)col * Ks + (w - K)] ^= m[k];
                }
              }
            }
          for (u32 k = 0; k < nw; ++k) {
            const u32 w = w0 + k * Lw;
            if (w < L) { s_c0[sl * L + w] = a0[k]; s_c1[sl * L + w] = a1[k]; }
          }
        }
        __syncthreads();
        // (3) add the slices' counters (mod 4); the sum must be even; the
        // phase bit joins the constant term of each masked stabilizer row
        for (u32 w = tid; w < L; w += T) {
          const u64 mw = s_m[w];
          if (!mw) continue;
          u64 s0 = 0, s1 = 0;
          for (u32 r = 0; r < S; ++r) {
            const u64 b0 = s_c0[r * L + w], b1 = s_c1[r * L + w];
            const u64 carry = s0 & b0;
            s0 ^= b0;
            s1 ^= b1 ^ carry;
          }
          if (s0 & mw) atomicOr(&s_flags, 1u);
          if (w >= K) sgc[w - K] ^= mw & s1;
        }
        __syncthreads();
        // (4) D_p <- S_p, S_p <- Z_q; clear S_p's old sign vector
        for (u32 j = tid; j < n; j += T) {
          const u64 xb = (s_px[j >> 6] >> (j & 63u)) & 1ULL, zb = (s_pz[j >> 6] >> (j & 63u)) & 1ULL;
          u64 *x = X + (size_t)j * Ls;
          u64 *z = Z + (size_t)j * Ls;
          x[wd] = (x[wd] & ~bit) | (xb ? bit : 0ULL);
          z[wd] = (z[wd] & ~bit) | (zb ? bit : 0ULL);
          x[ws] &= ~bit;
          z[ws] = (z[ws] & ~bit) | ((j == q) ? bit : 0ULL);
        }
        for (u32 v = tid; v <= i; v += T) {
          if ((s_sgn[v >> 6] >> (v & 63u)) & 1ULL) {
            const u32 col = (v == i) ? count : v;
            sg[(size_t)col * Ks + wd] &= ~bit;
          }
        }
        __syncthreads();
        // (5) S_p's sign is coin i
        if (tid == 0) {
          sg[(size_t)i * Ks + wd] |= bit;
          d.kind[i] = 1;
        }
        __syncthreads();
      } else {
        // ------------------------------------------------ deterministic case
        for (u32 w = tid; w < K; w += T) s_px[w] = colq[w];  // A mask (destabilizer half)
        __syncthreads();
        int acc = 0;
        u32 bad = 0;
        for (u32 j = tid; j < n; j += T) {
          const u64 *xc = X + (size_t)j * Ls + K;
          const u64 *zc = Z + (size_t)j * Ls + K;
          u64 cx = 0, cz = 0;  // all-ones when the running product has x (z) on column j
          for (u32 w = 0; w < K; ++w) {
            const u64 a = s_px[w];
            if (!a) continue;
            const u64 sx = xc[w] & a, sz = zc[w] & a;
            u64 ex = sx, ez = sz;
            ex ^= ex << 1; ex ^= ex << 2; ex ^= ex << 4; ex ^= ex << 8; ex ^= ex << 16; ex ^= ex << 32;
            ez ^= ez << 1; ez ^= ez << 2; ez ^= ez << 4; ez ^= ez << 8; ez ^= ez << 16; ez ^= ez << 32;
            ex = (ex << 1) ^ cx;
            ez = (ez << 1) ^ cz;
            const u64 p_x = sx & ~sz, p_y = sx & sz, p_z = ~sx & sz;
            const u64 plus = (p_x & ex & ez) | (p_y & ~ex & ez) | (p_z & ex & ~ez);
            const u64 minus = (p_x & ~ex & ez) | (p_y & ex & ~ez) | (p_z & ex & ez);
            acc += __popcll(plus) - __popcll(minus);
            if (__popcll(sx) & 1) cx = ~cx;
            if (__popcll(sz) & 1) cz = ~cz;
          }
          if (cx != 0 || (cz != 0) != (j == q)) bad = 1;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) s_acc[wave] = acc;
        if (bad) atomicOr(&s_flags, 2u);
        __syncthreads();
        int e = 0;
        for (u32 v = 0; v < nwaves; ++v) e += s_acc[v];
        // affine form: XOR over A of the sign vectors, constant gets bit 1 of e
        for (u32 vb = 0; vb <= i; vb += T) {
          const u32 v = vb + tid;
          u32 par = 0;
          if (v <= i) {
            const u32 col = (v == i) ? count : v;
            const u64 *c = sg + (size_t)col * Ks;
            for (u32 w = 0; w < K; ++w) par ^= (u32)__popcll(c[w] & s_px[w]) & 1u;
          }
          if (v == i) {
            if (e & 1) atomicOr(&s_flags, 1u);
            d.fc[i] = (uint8_t)(par ^ (((u32)e >> 1) & 1u));
            d.kind[i] = 0;
          }
          const u64 bb = __ballot(v < i && par);
          if (lane == 0 && v <= i) d.fm[(size_t)i * CW + (v >> 6)] = bb;
        }
        __syncthreads();
      }
    }

    // ---- shots: coins and outcome words
    for (u32 s = tid; s < d.shots; s += T) {
      u64 *cb = d.coinbuf + (size_t)s * CW;
      u64 *out = d.out + (size_t)s * CW;
      for (u32 ow = 0; ow < CW; ++ow) {
        u64 c = 0;
        const u32 i0 = ow * 64u;
        for (u32 k = 0; k < 64u && i0 + k < count; ++k)
          c |= (u64)coin_bit(d.seed, d.shot_begin + s, d.meas_base + i0 + k) << k;
        cb[ow] = c;
        u64 word = c;
        for (u32 k = 0; k < 64u && i0 + k < count; ++k) {
          const u32 i = i0 + k;
          if (d.kind[i]) continue;
          u32 par = d.fc[i];
          const u64 *f = d.fm + (size_t)i * CW;
          for (u32 u = 0; u <= ow; ++u) par ^= (u32)__popcll(f[u] & cb[u]) & 1u;
          word = (word & ~(1ULL << k)) | ((u64)(par & 1u) << k);
        }
        out[ow] = word;
      }
    }
    __syncthreads();
    if (tid == 0 && s_flags) atomicOr(d.flags, s_flags);
    __syncthreads();
  }
}

hipError_t launch_batch(const BatchItem *items, u32 nitems, u32 *next, u32 block, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(block), 0, s, items, nitems, next);
  return hipGetLastError();
}

}  // namespace sq
