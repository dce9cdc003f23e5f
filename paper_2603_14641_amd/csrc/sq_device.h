// Device helpers shared by the kernel files: wave64 lane masks, 16-byte
// word-pair loads and stores, and the counter-based coin generator.
#pragma once
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

// Streaming forms for tableau columns, which a pass reads and writes once
// and which far exceed the caches: the accesses carry the non-temporal hint.
template <int WPT>
__device__ __forceinline__ void ldw_nt(const u64 *p, u64 (&v)[WPT]) {
  if constexpr (WPT == 2) {
    const u64x2 t = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(p));
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = __builtin_nontemporal_load(p);
  }
}

template <int WPT>
__device__ __forceinline__ void stw_nt(u64 *p, const u64 (&v)[WPT]) {
  if constexpr (WPT == 2) {
    u64x2 t;
    t.x = v[0];
    t.y = v[1];
    __builtin_nontemporal_store(t, reinterpret_cast<u64x2 *>(p));
  } else {
    __builtin_nontemporal_store(v[0], p);
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

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

// 64-bit xor-shuffle across the wave, as two 32-bit shuffles.
__device__ __forceinline__ u64 shfl_xor_u64(u64 v, int off) {
  const u32 lo = (u32)__shfl_xor((int)(u32)v, off), hi = (u32)__shfl_xor((int)(u32)(v >> 32), off);
  return ((u64)hi << 32) | lo;
}

// a ^ (b & m) with a 32-bit mask m applied to both halves, one v_bitop3_b32
// per half. The immediate is the truth table: the function evaluated on the
// bit patterns 0xF0, 0xCC, 0xAA standing for the first, second and third
// operand (0xF0 ^ (0xCC & 0xAA) = 0x78).
__device__ __forceinline__ u64 xor_and(u64 a, u64 b, u32 m) {
  const u32 lo = __builtin_amdgcn_bitop3_b32((u32)a, (u32)b, m, 0x78);
  const u32 hi = __builtin_amdgcn_bitop3_b32((u32)(a >> 32), (u32)(b >> 32), m, 0x78);
  return ((u64)hi << 32) | lo;
}

// Transpose of a 64 x 64 bit tile held one word per lane: on return lane l
// holds the word whose bit b is bit l of lane b's input word. Six butterfly
// steps exchange blocks of 32, 16, ... 1 bits between lanes l and l ^ j
// (the bit-group shuffle with masks 0x00000000FFFFFFFF ... 0x5555...).
// Every lane of the wave must take part.
__device__ __forceinline__ u64 transpose64(u64 v) {
  const u32 lane = threadIdx.x & 63u;
  const u64 masks[6] = {0x00000000FFFFFFFFULL, 0x0000FFFF0000FFFFULL, 0x00FF00FF00FF00FFULL,
                        0x0F0F0F0F0F0F0F0FULL, 0x3333333333333333ULL, 0x5555555555555555ULL};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const u32 j = 32u >> k;
    const u64 other = shfl_xor_u64(v, (int)j);
    if ((lane & j) == 0) {
      const u64 t = ((v >> j) ^ other) & masks[k];
      v ^= t << j;
    } else {
      const u64 t = ((other >> j) ^ v) & masks[k];
      v ^= t;
    }
  }
  return v;
}

// 64-bit broadcast of lane src's value, as two 32-bit shuffles.
__device__ __forceinline__ u64 shfl_u64(u64 v, int src) {
  const u32 lo = (u32)__shfl((int)(u32)v, src), hi = (u32)__shfl((int)(u32)(v >> 32), src);
  return ((u64)hi << 32) | lo;
}

}  // namespace sq
