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
// The sweep itself uses the measurement kernels of sq_measure.hip in their
// symbolic mode (SymCtx); this file holds the set-up and the per-shot
// evaluation.
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
