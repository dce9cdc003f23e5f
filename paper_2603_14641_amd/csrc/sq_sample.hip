// Shot sampling by one symbolic measurement sweep.
//
// Shot s of a measured qubit list is, by definition, the outcome string that
// the CHP measurement sequence gives on a copy of the tableau when
// measurement j draws coin c_j(s) = coin(seed, shot_begin + s, meas_base + j).
// Two facts make one sweep serve every shot:
//   * the x/z bits (hence every pivot, mask and random/deterministic
//     decision) never depend on signs, so they evolve identically in all shots;
//   * every stabilizer sign stays an affine GF(2) function of the coins:
//     rowsum XORs the pivot's sign (plus a phase bit that depends on x/z
//     only), a random measurement sets the pivot's sign to its own coin, and a
//     deterministic outcome is the XOR of the signs of the stabilizers in A
//     plus a phase bit.
// Destabilizer signs never feed back into stabilizer signs, so they are not
// tracked. Sign column v (v < count: coefficient of coin v; v = count: the
// constant term) holds one bit per stabilizer row, K words, stride Ks.
#include "sq_device.h"

namespace sq {

// Constant column <- stabilizer signs of the tableau; coin columns <- 0.
__global__ void k_sample_init(const u64 *__restrict__ R, u64 *__restrict__ sg, u32 K, u32 Ks, u32 count) {
  const size_t total = (size_t)(count + 1) * Ks;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const size_t v = i / Ks, w = i % Ks;
    sg[i] = (v == count && w < K) ? R[K + w] : 0ULL;
  }
}

// Compact the sign columns in which the pivot stabilizer S_p has a 1:
// candidates are the coins of the earlier measurements (v < i) and the
// constant (v = count).
__global__ void k_gather_signs(const u64 *__restrict__ sg, MeasState *__restrict__ st, u32 *__restrict__ svlist,
                               u32 Ks, u32 i, u32 count) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
  u32 v = 0, bit = 0;
  if (t <= i) {
    v = (t == i) ? count : t;
    bit = (u32)(sg[(size_t)v * Ks + ((u32)p >> 6)] >> ((u32)p & 63u)) & 1u;
  }
  const u64 b = __ballot(bit);
  u32 base = 0;
  if ((threadIdx.x & 63u) == 0 && b) base = atomicAdd(&st->nsv, (u32)__popcll(b));
  base = (u32)__shfl((int)base, 0);
  if (bit) svlist[base + (u32)__popcll(b & lanemask_lt())] = v;
}

// Every masked stabilizer row takes S_p's sign vector: sg[v] ^= mask_S for
// each listed column v. Grid: (row-word tiles, column chunks).
__global__ void k_signcols(u64 *__restrict__ sg, const u64 *__restrict__ mask, const MeasState *__restrict__ st,
                           const u32 *__restrict__ svlist, u32 K, u32 Ks,
                           u32 vpc) {
  if (st->p < 0) return;
  const u32 nsv = st->nsv;
  const u32 v0 = blockIdx.y * vpc;
  if (v0 >= nsv) return;
  const u32 v1 = min(v0 + vpc, nsv);
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= K) return;
  const u64 m = mask[K + w];
  if (m == 0) return;
  for (u32 k = v0; k < v1; ++k) {
    u64 *c = sg + (size_t)svlist[k] * Ks + w;
    *c ^= m;
  }
}

// Random case, after the rowsum pass and k_signcols: add the phase bit of each
// masked stabilizer row to the constant column (the chunk counters hold the
// g sum mod 4, which must be even); D_p <- S_p and S_p <- Z_q in x/z; S_p's
// sign vector becomes (0..., coin i, ...): its constant bit is cleared here,
// its other bits by k_spvec.
__global__ void k_finalize_sym(u64 *__restrict__ X, u64 *__restrict__ Z, u64 *__restrict__ sgc,
                               const u64 *__restrict__ mask, const u64 *__restrict__ pivx, const u64 *__restrict__ pivz,
                               const u64 *__restrict__ cnt0, const u64 *__restrict__ cnt1, MeasState *__restrict__ st,
                               u32 Ls, u32 K, u32 n, u32 q, u32 cpc) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 tid = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 wd = (u32)p >> 6;
  const u64 bit = 1ULL << ((u32)p & 63u);
  if (tid < K) {
    const u32 w = tid;
    const u64 m = mask[K + w];
    u64 c = sgc[w];
    bool touched = false;
    if (m != 0) {
      const u32 nch = (st->ncols + cpc - 1) / cpc;
      u64 s0 = 0, s1 = 0;
      for (u32 ch = 0; ch < nch; ++ch) {
        const u64 b0 = cnt0[(size_t)ch * Ls + K + w], b1 = cnt1[(size_t)ch * Ls + K + w];
        const u64 carry = s0 & b0;
        s0 ^= b0;
        s1 ^= b1 ^ carry;
      }
      if (s0 & m) atomicOr(&st->flags, 1u);
      c ^= m & s1;
      touched = true;
    }
    if (w == wd) {
      c &= ~bit;
      touched = true;
    }
    if (touched) sgc[w] = c;
  }
  if (tid < n) {
    const u32 j = tid;
    const u64 xb = (pivx[j >> 6] >> (j & 63u)) & 1ULL, zb = (pivz[j >> 6] >> (j & 63u)) & 1ULL;
    u64 *x = X + (size_t)j * Ls;
    u64 *z = Z + (size_t)j * Ls;
    const u32 ws = K + wd;
    x[wd] = (x[wd] & ~bit) | (xb ? bit : 0ULL);
    z[wd] = (z[wd] & ~bit) | (zb ? bit : 0ULL);
    x[ws] &= ~bit;
    z[ws] = (z[ws] & ~bit) | ((j == q) ? bit : 0ULL);
  }
}

// S_p's coin coefficients: clear every listed coin column at p, set column i.
__global__ void k_spvec(u64 *__restrict__ sg, const MeasState *__restrict__ st, const u32 *__restrict__ svlist, uint8_t *__restrict__ kind, u32 Ks, u32 i, u32 count) {
  const int32_t p = st->p;
  if (p < 0) return;
  const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 wd = (u32)p >> 6;
  const u64 bit = 1ULL << ((u32)p & 63u);
  if (t < st->nsv) {
    const u32 v = svlist[t];
    if (v != count) sg[(size_t)v * Ks + wd] &= ~bit;
  }
  if (t == 0) {
    sg[(size_t)i * Ks + wd] |= bit;
    kind[i] = 1;
  }
}

// Deterministic case: the outcome's affine form is the XOR over A of the
// stabilizers' sign vectors, plus bit 1 of the phase sum in the constant.
// One lane per candidate column v (coins 0..i-1, then the constant).
__global__ void k_detfinal_sym(const u64 *__restrict__ sg, const u64 *__restrict__ mask, MeasState *__restrict__ st,
                               uint8_t *__restrict__ kind, u64 *__restrict__ fm, uint8_t *__restrict__ fc, u32 K,
                               u32 Ks, u32 CW, u32 i, u32 count) {
  if (st->p >= 0) return;
  const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
  u32 par = 0;
  if (t <= i) {
    const u32 v = (t == i) ? count : t;
    const u64 *c = sg + (size_t)v * Ks;
    for (u32 w = 0; w < K; ++w) par ^= (u32)__popcll(c[w] & mask[w]) & 1u;
  }
  if (t == i) {
    const u32 e = st->det_acc & 3u;
    if (e & 1u) atomicOr(&st->flags, 1u);
    fc[i] = (uint8_t)(par ^ (e >> 1));
    kind[i] = 0;
  }
  // coin coefficients: lanes t < i, packed 64 per word by ballot; every word
  // up to i/64 is written (bits of later coins are 0)
  const u64 b = __ballot(t < i && par);
  if ((threadIdx.x & 63u) == 0 && t <= i) fm[(size_t)i * CW + (t >> 6)] = b;
}

// Coin bits of every (shot, measurement): cw[s*CW + j/64] bit j%64.
__global__ void k_coins(u64 *__restrict__ cw, u64 seed, u64 shot_begin, u64 meas_base, u32 shots, u32 count,
                        u32 CW) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)shots * CW) return;
  const u32 s = (u32)(idx / CW), wd = (u32)(idx % CW);
  u64 word = 0;
  const u32 j0 = wd * 64u;
  for (u32 k = 0; k < 64u && j0 + k < count; ++k)
    word |= (u64)coin_bit(seed, shot_begin + s, meas_base + j0 + k) << k;
  cw[idx] = word;
}

// Outcome word (s, ow): random outcomes are their coins; deterministic ones
// evaluate their affine form on the shot's coins.
__global__ void k_eval(const u64 *__restrict__ cw, const uint8_t *__restrict__ kind, const u64 *__restrict__ fm,
                       const uint8_t *__restrict__ fc, u64 *__restrict__ out, u32 shots, u32 count, u32 CW) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)shots * CW) return;
  const u32 s = (u32)(idx / CW), ow = (u32)(idx % CW);
  const u64 *c = cw + (size_t)s * CW;
  u64 word = c[ow];
  const u32 i0 = ow * 64u;
  for (u32 k = 0; k < 64u && i0 + k < count; ++k) {
    const u32 i = i0 + k;
    if (kind[i]) continue;
    u32 par = fc[i];
    const u64 *f = fm + (size_t)i * CW;
    for (u32 u = 0; u <= (i >> 6); ++u) par ^= (u32)__popcll(f[u] & c[u]) & 1u;
    word = (word & ~(1ULL << k)) | ((u64)(par & 1u) << k);
  }
  if (i0 + 64u > count) word &= (count > i0) ? ((~0ULL) >> (64u - (count - i0))) : 0ULL;
  out[idx] = word;
}

// Launchers.
hipError_t launch_sample_init(const TabDev &t, u64 *sg, u32 Ks, u32 count, hipStream_t s) {
  const size_t total = (size_t)(count + 1) * Ks;
  const u32 blocks = (u32)std::min<u64>(cdiv(total, 256), 65536);
  hipLaunchKernelGGL(k_sample_init, dim3(blocks), dim3(256), 0, s, t.R, sg, t.K, Ks, count);
  return hipGetLastError();
}

hipError_t launch_gather_signs(const u64 *sg, MeasState *st, u32 *svlist, u32 Ks, u32 i, u32 count,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_gather_signs, dim3(cdiv(i + 1, 256)), dim3(256), 0, s, sg, st, svlist, Ks, i, count);
  return hipGetLastError();
}

hipError_t launch_signcols(const TabDev &t, u64 *sg, const u64 *mask, const MeasState *st, const u32 *svlist, u32 Ks,
                           u32 max_v, hipStream_t s) {
  const u32 vpc = 32;
  dim3 grid(cdiv(t.K, 256), std::max<u32>(1, cdiv(max_v, vpc)));
  hipLaunchKernelGGL(k_signcols, grid, dim3(256), 0, s, sg, mask, st, svlist, t.K, Ks, vpc);
  return hipGetLastError();
}

hipError_t launch_finalize_sym(const TabDev &t, u32 q, u64 *sgc, const u64 *mask, const u64 *pivx, const u64 *pivz,
                               const u64 *cnt0, const u64 *cnt1, MeasState *st, u32 cpc, hipStream_t s) {
  const u32 threads = std::max(t.K, t.n);
  hipLaunchKernelGGL(k_finalize_sym, dim3(cdiv(threads, 256)), dim3(256), 0, s, t.X, t.Z, sgc, mask, pivx, pivz,
                     cnt0, cnt1, st, t.Ls, t.K, t.n, q, cpc);
  return hipGetLastError();
}

hipError_t launch_spvec(u64 *sg, const MeasState *st, const u32 *svlist, uint8_t *kind,
                        u32 Ks, u32 i, u32 count, hipStream_t s) {
  hipLaunchKernelGGL(k_spvec, dim3(cdiv(i + 1, 256)), dim3(256), 0, s, sg, st, svlist, kind, Ks, i, count);
  return hipGetLastError();
}

hipError_t launch_detfinal_sym(const TabDev &t, const u64 *sg, const u64 *mask, MeasState *st, uint8_t *kind,
                               u64 *fm, uint8_t *fc, u32 Ks, u32 CW, u32 i, u32 count, hipStream_t s) {
  hipLaunchKernelGGL(k_detfinal_sym, dim3(cdiv(i + 1, 256)), dim3(256), 0, s, sg, mask, st, kind, fm, fc, t.K, Ks,
                     CW, i, count);
  return hipGetLastError();
}

hipError_t launch_coins(u64 *cw, u64 seed, u64 shot_begin, u64 meas_base, u32 shots, u32 count, u32 CW,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_coins, dim3(cdiv((u64)shots * CW, 256)), dim3(256), 0, s, cw, seed, shot_begin, meas_base,
                     shots, count, CW);
  return hipGetLastError();
}

hipError_t launch_eval(const u64 *cw, const uint8_t *kind, const u64 *fm, const uint8_t *fc, u64 *out, u32 shots,
                       u32 count, u32 CW, hipStream_t s) {
  hipLaunchKernelGGL(k_eval, dim3(cdiv((u64)shots * CW, 256)), dim3(256), 0, s, cw, kind, fm, fc, out, shots, count,
                     CW);
  return hipGetLastError();
}

}  // namespace sq
