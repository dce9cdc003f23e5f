// Pauli-frame sampling (the paper's "Sampling" section, Algorithm
// alg:sampling): many shots of a compiled program without collapsing a
// tableau per shot. Frames are stored like tableau columns with shots in
// place of rows: Fx[q * Ls + w], Fz[q * Ls + w], bit b = shot 64 w + b. Gate
// passes reuse the tableau gate kernel (a frame transforms like a tableau
// row; its sign is not used). A measurement of qubit q records the x word and
// draws the z word afresh; the outcome is the reference sample's bit XOR the
// recorded frame bit.
//
// Random words: word w of event e is output word 0 of Philox4x64-10 with key
// (seed, 2^63 + w) and counter (e, 0, 0, 0); bit b belongs to shot 64 w + b.
// Events 0..n-1 initialise z of each qubit; event n + i re-draws z after
// measurement i.
#include "sq_device.h"

namespace sq {

constexpr u64 FRAME_KEY = 1ULL << 63;

__global__ void k_frame_init(u64 *__restrict__ Fx, u64 *__restrict__ Fz, u32 n, u32 Lf, u32 Ls, u64 seed) {
  const u64 idx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (u64)n * Lf) return;
  const u32 q = (u32)(idx / Lf), w = (u32)(idx % Lf);
  Fx[(size_t)q * Ls + w] = 0;
  Fz[(size_t)q * Ls + w] = philox_word0(q, 0, 0, 0, seed, FRAME_KEY + w);
}

// Thread per shot word; the segment's measurements in program order (a qubit
// measured twice must see its own re-draw).
__global__ void k_frame_measure(const u64 *__restrict__ Fx, u64 *__restrict__ Fz, const u32 *__restrict__ qubits,
                                u32 count, u64 m0, const uint8_t *__restrict__ ref, u64 *__restrict__ rec, u32 n,
                                u32 Lf, u32 Ls, u64 seed) {
  const u32 w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= Lf) return;
  for (u32 i = 0; i < count; ++i) {
    const u64 m = m0 + i;
    const u32 q = qubits[m];
    rec[(size_t)m * Lf + w] = Fx[(size_t)q * Ls + w] ^ (ref[m] ? ~0ULL : 0ULL);
    Fz[(size_t)q * Ls + w] = philox_word0((u64)n + m, 0, 0, 0, seed, FRAME_KEY + w);
  }
}

// Records (measurement-major, one word per 64 shots) to the shot-major
// output: a wave takes 64 measurements x 64 shots, lane l loads measurement
// 64 t + l, and six butterfly steps (swap the off-diagonal halves of ever
// smaller blocks between lanes l and l ^ j) leave lane l with shot 64 w + l.
__global__ __launch_bounds__(256) void k_frame_transpose(const u64 *__restrict__ rec, u64 *__restrict__ out, u64 M,
                                                         u32 W, u32 Lf, u32 shots) {
  const u32 lane = threadIdx.x & 63u;
  const u64 tile = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // (measurement word, shot word)
  const u32 iw = (u32)(tile % W), w = (u32)(tile / W);
  if (w >= Lf) return;  // uniform over the wave
  const u64 m = (u64)iw * 64u + lane;
  const u64 v = transpose64(m < M ? rec[m * Lf + w] : 0ULL);
  const u64 s = (u64)w * 64u + lane;
  if (s < shots) out[s * W + iw] = v;
}

hipError_t launch_frame_init(u64 *Fx, u64 *Fz, u32 n, u32 Lf, u32 Ls, u64 seed, hipStream_t s) {
  const u64 total = (u64)n * Lf;
  hipLaunchKernelGGL(k_frame_init, dim3((u32)((total + 255) / 256)), dim3(256), 0, s, Fx, Fz, n, Lf, Ls, seed);
  return hipGetLastError();
}

hipError_t launch_frame_measure(const u64 *Fx, u64 *Fz, const u32 *qubits, u32 count, u64 m0, const uint8_t *ref,
                                u64 *rec, u32 n, u32 Lf, u32 Ls, u64 seed, hipStream_t s) {
  hipLaunchKernelGGL(k_frame_measure, dim3(cdiv(Lf, 256)), dim3(256), 0, s, Fx, Fz, qubits, count, m0, ref, rec, n,
                     Lf, Ls, seed);
  return hipGetLastError();
}

hipError_t launch_frame_transpose(const u64 *rec, u64 *out, u64 M, u32 W, u32 Lf, u32 shots, hipStream_t s) {
  const u64 waves = (u64)W * Lf;
  hipLaunchKernelGGL(k_frame_transpose, dim3((u32)((waves * 64 + 255) / 256)), dim3(256), 0, s, rec, out, M, W, Lf,
                     shots);
  return hipGetLastError();
}

}  // namespace sq
