// Initialisation and canonical row-major export/import.
#include "sq_device.h"

namespace sq {

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

// Launchers.
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
