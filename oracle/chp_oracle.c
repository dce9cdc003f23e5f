/*
 * CPU oracle for the stabilizer-tableau simulator -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, row-major implementation of the CHP algorithm (Aaronson and
 * Gottesman's destabilizer tableau, as summarised in the paper's sections
 * "Tableau Formalism" and "The CHP algorithm"). It exists to check the GPU
 * library bit for bit. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the GPU library.
 *
 * Tableau: rows 0..n-1 are the destabilizers D_i, rows n..2n-1 the
 * stabilizers S_i. Row g holds bits x_gj, z_gj (j = qubit) packed LSB-first
 * into W = ceil(n/64) words each, and a sign bit r_g: the row is the Pauli
 * string (-1)^r_g * P_1 ... P_n with P_j = I, X, Z, Y for (x, z) = (0,0),
 * (1,0), (0,1), (1,1) (encoding of the "Tableau Formalism" section).
 *
 * A handle may hold only a subset of the 2n rows (for sampled checks at large
 * n). Gates act on every row independently, so a subset evolves exactly. A
 * measurement is decided on a subset only when its pivot lies inside a held
 * prefix S_0..S_{k-1} of stabilizer rows (see sqo_run); otherwise the run stops.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
  SQO_I = 0, SQO_H = 1, SQO_S = 2, SQO_SDG = 3, SQO_X = 4, SQO_Y = 5, SQO_Z = 6,
  SQO_CX = 7, SQO_CZ = 8, SQO_CY = 9, SQO_SWAP = 10, SQO_ISWAP = 11, SQO_MEASURE = 15
};

typedef struct {
  uint32_t n;        /* qubits */
  uint32_t W;        /* words per x (or z) half of a row */
  uint32_t nrows;    /* rows held */
  uint32_t *gid;     /* global row index of each held row */
  int32_t *local;    /* global row index -> held position, or -1 (2n entries) */
  uint64_t *x, *z;   /* nrows * W words */
  uint8_t *r;        /* nrows sign bits */
  uint64_t odd;      /* count of rowsums whose phase exponent was odd (must stay 0) */
  uint64_t badscratch; /* count of deterministic products that were not +-Z_q */
  uint64_t det_phase2; /* deterministic outcomes whose summed phase exponents were 2 mod 4 */
} sqo_tab;

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): a 4-word counter and 2-word key; each of the 10
 * rounds multiplies words 0 and 2 by fixed odd constants, crosses the high
 * halves into the other words with the round key, and the key is advanced by
 * two Weyl constants between rounds. */
#define SQO_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define SQO_PHILOX_M1 0xCA5A826395121157ULL
#define SQO_PHILOX_W0 0x9E3779B97F4A7C15ULL
#define SQO_PHILOX_W1 0xBB67AE8584CAA73BULL

void sqo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += SQO_PHILOX_W0; k1 += SQO_PHILOX_W1; }
    unsigned __int128 p0 = (unsigned __int128)SQO_PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)SQO_PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Outcome coin of measurement number m of shot `shot`: bit 0 of output word 0
 * with counter (m, 0, 0, 0) and key (seed, shot). */
int sqo_coin(uint64_t seed, uint64_t shot, uint64_t m) {
  uint64_t ctr[4] = {m, 0, 0, 0}, key[2] = {seed, shot}, out[4];
  sqo_philox4x64_10(ctr, key, out);
  return (int)(out[0] & 1);
}

/* ------------------------------------------------------------------ */
static inline int getb(const uint64_t *v, uint32_t j) { return (int)((v[j >> 6] >> (j & 63)) & 1); }
static inline void putb(uint64_t *v, uint32_t j, int b) {
  uint64_t m = 1ULL << (j & 63);
  if (b) v[j >> 6] |= m; else v[j >> 6] &= ~m;
}

/* Conjugate one row by one gate: P -> U P U^dagger. All right-hand sides use
 * the values before the gate. H, S and CX are the rules printed in the
 * "Tableau Formalism" section; the others follow by conjugation:
 * S^dagger = S^3, X P X flips the sign of Z and Y, Z P Z flips X and Y,
 * Y P Y flips X and Z, and CZ(a,b) = H_b CX(a,b) H_b. The remaining gates of
 * the paper's gate set are products of these, conjugated factor by factor in
 * time order: CY(a,b) = S_b CX(a,b) S_b^dagger (S^dagger first),
 * iSWAP(a,b) = SWAP CZ (S_a S_b) (the S gates first); SWAP exchanges the two
 * qubits' bits and leaves the sign. */
static void gate_on_row(uint64_t *x, uint64_t *z, uint8_t *r, uint32_t type, uint32_t a, uint32_t b) {
  if (type == SQO_CY) {
    gate_on_row(x, z, r, SQO_SDG, b, 0);
    gate_on_row(x, z, r, SQO_CX, a, b);
    gate_on_row(x, z, r, SQO_S, b, 0);
    return;
  }
  if (type == SQO_ISWAP) {
    gate_on_row(x, z, r, SQO_S, a, 0);
    gate_on_row(x, z, r, SQO_S, b, 0);
    gate_on_row(x, z, r, SQO_CZ, a, b);
    gate_on_row(x, z, r, SQO_SWAP, a, b);
    return;
  }
  int xa = getb(x, a), za = getb(z, a);
  switch (type) {
    case SQO_H:
      *r ^= (uint8_t)(xa & za);
      putb(x, a, za);
      putb(z, a, xa);
      break;
    case SQO_S:
      *r ^= (uint8_t)(xa & za);
      putb(z, a, za ^ xa);
      break;
    case SQO_SDG:
      *r ^= (uint8_t)(xa & (za ^ 1));
      putb(z, a, za ^ xa);
      break;
    case SQO_X:
      *r ^= (uint8_t)za;
      break;
    case SQO_Y:
      *r ^= (uint8_t)(xa ^ za);
      break;
    case SQO_Z:
      *r ^= (uint8_t)xa;
      break;
    case SQO_CX: {
      int xb = getb(x, b), zb = getb(z, b);
      *r ^= (uint8_t)(xa & zb & (xb ^ za ^ 1));
      putb(x, b, xb ^ xa);
      putb(z, a, za ^ zb);
      break;
    }
    case SQO_CZ: {
      int xb = getb(x, b), zb = getb(z, b);
      *r ^= (uint8_t)(xa & xb & (za ^ zb));
      putb(z, a, za ^ xb);
      putb(z, b, zb ^ xa);
      break;
    }
    case SQO_SWAP: {
      int xb = getb(x, b), zb = getb(z, b);
      putb(x, a, xb);
      putb(z, a, zb);
      putb(x, b, xa);
      putb(z, b, za);
      break;
    }
    default:
      break;
  }
}

/* g(x1,z1,x2,z2): the exponent of i in the product P1*P2 of single-qubit
 * Paulis (Aaronson-Gottesman): 0 for P1 = I; z2 - x2 for P1 = Y;
 * z2 (2 x2 - 1) for P1 = X; x2 (1 - 2 z2) for P1 = Z. */
int sqo_g(int x1, int z1, int x2, int z2) {
  if (!x1 && !z1) return 0;
  if (x1 && z1) return z2 - x2;
  if (x1) return z2 * (2 * x2 - 1);
  return x2 * (1 - 2 * z2);
}

/* The same function summed over the 64 bit positions of one word, mod 4:
 * +1 where (P1,P2) is (X,Y), (Y,Z) or (Z,X); -1 where it is (X,Z), (Y,X) or
 * (Z,Y); 0 elsewhere. */
int sqo_gsum_word(uint64_t x1, uint64_t z1, uint64_t x2, uint64_t z2) {
  uint64_t p_x = x1 & ~z1, p_y = x1 & z1, p_z = ~x1 & z1;
  uint64_t plus = (p_x & x2 & z2) | (p_y & ~x2 & z2) | (p_z & x2 & ~z2);
  uint64_t minus = (p_x & ~x2 & z2) | (p_y & x2 & ~z2) | (p_z & x2 & z2);
  int d = __builtin_popcountll(plus) - __builtin_popcountll(minus);
  return ((d % 4) + 4) % 4;
}

/* rowsum(h, i): row h <- P_i * P_h. The phase exponent
 * e = 2 r_h + 2 r_i + sum_j g(x_ij, z_ij, x_hj, z_hj) (mod 4) must be 0 or 2;
 * r_h <- e / 2. Returns 1 if e was odd (an error: the product is not
 * Hermitian). If gsum is not NULL, the g sum (mod 4) is added to it. */
static int row_mul_g(uint64_t *xh, uint64_t *zh, uint8_t *rh,
                     const uint64_t *xi, const uint64_t *zi, uint8_t ri, uint32_t W, int *gsum) {
  int g = 0;
  for (uint32_t w = 0; w < W; ++w) g += sqo_gsum_word(xi[w], zi[w], xh[w], zh[w]);
  if (gsum) *gsum = (*gsum + g) & 3;
  int e = 2 * (int)*rh + 2 * (int)ri + g;
  e &= 3;
  for (uint32_t w = 0; w < W; ++w) { xh[w] ^= xi[w]; zh[w] ^= zi[w]; }
  *rh = (uint8_t)(e >> 1);
  return e & 1;
}

static int row_mul(uint64_t *xh, uint64_t *zh, uint8_t *rh,
                   const uint64_t *xi, const uint64_t *zi, uint8_t ri, uint32_t W) {
  return row_mul_g(xh, zh, rh, xi, zi, ri, W, NULL);
}

/* ------------------------------------------------------------------ */
static uint64_t *ROWX(sqo_tab *t, uint32_t k) { return t->x + (size_t)k * t->W; }
static uint64_t *ROWZ(sqo_tab *t, uint32_t k) { return t->z + (size_t)k * t->W; }

static void init_row(sqo_tab *t, uint32_t k) {
  uint32_t g = t->gid[k];
  memset(ROWX(t, k), 0, sizeof(uint64_t) * t->W);
  memset(ROWZ(t, k), 0, sizeof(uint64_t) * t->W);
  t->r[k] = 0;
  if (g < t->n) putb(ROWX(t, k), g, 1);          /* D_g = +X_g */
  else putb(ROWZ(t, k), g - t->n, 1);            /* S_i = +Z_i */
}

/* Create a handle holding the given global rows (NULL: all 2n rows), in
 * the state |0...0>: D_i = +X_i, S_i = +Z_i. */
sqo_tab *sqo_create(uint32_t n, const uint32_t *rows, uint32_t nrows) {
  if (n == 0) return NULL;
  sqo_tab *t = (sqo_tab *)calloc(1, sizeof(sqo_tab));
  if (!t) return NULL;
  t->n = n;
  t->W = (n + 63) / 64;
  t->nrows = rows ? nrows : 2 * n;
  t->gid = (uint32_t *)malloc(sizeof(uint32_t) * (t->nrows ? t->nrows : 1));
  t->local = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n);
  t->x = (uint64_t *)calloc((size_t)t->nrows * t->W + 1, sizeof(uint64_t));
  t->z = (uint64_t *)calloc((size_t)t->nrows * t->W + 1, sizeof(uint64_t));
  t->r = (uint8_t *)calloc(t->nrows + 1, 1);
  if (!t->gid || !t->local || !t->x || !t->z || !t->r) {
    free(t->gid); free(t->local); free(t->x); free(t->z); free(t->r); free(t);
    return NULL;
  }
  for (size_t g = 0; g < 2 * (size_t)n; ++g) t->local[g] = -1;
  for (uint32_t k = 0; k < t->nrows; ++k) {
    uint32_t g = rows ? rows[k] : k;
    if (g >= 2 * n || t->local[g] >= 0) {  /* out of range or repeated */
      free(t->gid); free(t->local); free(t->x); free(t->z); free(t->r); free(t);
      return NULL;
    }
    t->gid[k] = g;
    t->local[g] = (int32_t)k;
  }
  for (uint32_t k = 0; k < t->nrows; ++k) init_row(t, k);
  return t;
}

void sqo_destroy(sqo_tab *t) {
  if (!t) return;
  free(t->gid); free(t->local); free(t->x); free(t->z); free(t->r); free(t);
}

uint32_t sqo_words(const sqo_tab *t) { return t->W; }
uint32_t sqo_nrows(const sqo_tab *t) { return t->nrows; }
uint64_t sqo_odd_count(const sqo_tab *t) { return t->odd; }
uint64_t sqo_badscratch_count(const sqo_tab *t) { return t->badscratch; }
uint64_t sqo_det_phase2_count(const sqo_tab *t) { return t->det_phase2; }

/* Copy the held rows out (row k of the outputs is held row k). */
void sqo_get_rows(const sqo_tab *t, uint64_t *x, uint64_t *z, uint8_t *r) {
  memcpy(x, t->x, sizeof(uint64_t) * (size_t)t->nrows * t->W);
  memcpy(z, t->z, sizeof(uint64_t) * (size_t)t->nrows * t->W);
  memcpy(r, t->r, t->nrows);
}

void sqo_set_rows(sqo_tab *t, const uint64_t *x, const uint64_t *z, const uint8_t *r) {
  memcpy(t->x, x, sizeof(uint64_t) * (size_t)t->nrows * t->W);
  memcpy(t->z, z, sizeof(uint64_t) * (size_t)t->nrows * t->W);
  memcpy(t->r, r, t->nrows);
}

/* Apply rowsum(h, i) on held positions (exposed for brute-force checks). */
int sqo_rowsum(sqo_tab *t, uint32_t h, uint32_t i) {
  int odd = row_mul(ROWX(t, h), ROWZ(t, h), &t->r[h], ROWX(t, i), ROWZ(t, i), t->r[i], t->W);
  t->odd += (uint64_t)odd;
  return odd;
}

/* Apply gates ops[0..count) to every held row. Rows are independent under
 * gates, so each row takes the whole gate sequence in order. */
static void apply_gate_run(sqo_tab *t, const uint32_t *ops, size_t count) {
  #pragma omp parallel for schedule(dynamic, 1)
  for (long k = 0; k < (long)t->nrows; ++k) {
    uint64_t *x = ROWX(t, (uint32_t)k), *z = ROWZ(t, (uint32_t)k);
    uint8_t *r = &t->r[k];
    for (size_t o = 0; o < count; ++o)
      gate_on_row(x, z, r, ops[3 * o], ops[3 * o + 1], ops[3 * o + 2]);
  }
}

/* Length k of the held stabilizer prefix S_0..S_{k-1}. */
static uint32_t held_stab_prefix(const sqo_tab *t) {
  uint32_t k = 0;
  while (k < t->n && t->local[t->n + k] >= 0) ++k;
  return k;
}

/* Measure Z on qubit q (CHP, "The CHP algorithm" section, with Aaronson and
 * Gottesman's bit-level procedure):
 *   random case: p = the smallest i with x(S_i)_q = 1. Every row h other
 *   than D_p and S_p with x_hq = 1 gets rowsum(h, S_p); then D_p <- S_p and
 *   S_p <- (-1)^coin Z_q; the outcome is the coin.
 *   deterministic case: multiply, in ascending i, the stabilizers S_i whose
 *   destabilizer has x(D_i)_q = 1 into a scratch row that starts at +I; the
 *   product is +-Z_q and its sign bit is the outcome.
 * Returns the outcome, or -1 if the held rows cannot decide it. */
static int measure(sqo_tab *t, uint32_t q, int coin, int *was_random) {
  const uint32_t n = t->n;
  const uint32_t k = held_stab_prefix(t);
  int32_t p = -1;
  for (uint32_t i = 0; i < k; ++i) {
    if (getb(ROWX(t, (uint32_t)t->local[n + i]), q)) { p = (int32_t)i; break; }
  }
  if (p >= 0) {
    const uint32_t sp = (uint32_t)t->local[n + p];
    const int32_t dp = t->local[p];
    uint64_t odd = 0;
    #pragma omp parallel for schedule(static) reduction(+ : odd)
    for (long h = 0; h < (long)t->nrows; ++h) {
      if ((uint32_t)h == sp || (int32_t)h == dp) continue;
      if (!getb(ROWX(t, (uint32_t)h), q)) continue;
      odd += (uint64_t)row_mul(ROWX(t, (uint32_t)h), ROWZ(t, (uint32_t)h), &t->r[h],
                               ROWX(t, sp), ROWZ(t, sp), t->r[sp], t->W);
    }
    t->odd += odd;
    if (dp >= 0) {
      memcpy(ROWX(t, (uint32_t)dp), ROWX(t, sp), sizeof(uint64_t) * t->W);
      memcpy(ROWZ(t, (uint32_t)dp), ROWZ(t, sp), sizeof(uint64_t) * t->W);
      t->r[dp] = t->r[sp];
    }
    memset(ROWX(t, sp), 0, sizeof(uint64_t) * t->W);
    memset(ROWZ(t, sp), 0, sizeof(uint64_t) * t->W);
    putb(ROWZ(t, sp), q, 1);
    t->r[sp] = (uint8_t)coin;
    *was_random = 1;
    return coin;
  }
  if (k < n) return -1;               /* pivot may lie outside the held rows */
  for (uint32_t i = 0; i < n; ++i)
    if (t->local[i] < 0) return -1;   /* deterministic case needs every D row */
  uint64_t *sx = (uint64_t *)calloc(t->W, sizeof(uint64_t));
  uint64_t *sz = (uint64_t *)calloc(t->W, sizeof(uint64_t));
  uint8_t sr = 0;
  int gsum = 0;
  for (uint32_t i = 0; i < n; ++i) {
    if (!getb(ROWX(t, (uint32_t)t->local[i]), q)) continue;
    uint32_t s = (uint32_t)t->local[n + i];
    t->odd += (uint64_t)row_mul_g(sx, sz, &sr, ROWX(t, s), ROWZ(t, s), t->r[s], t->W, &gsum);
  }
  if (gsum == 2) t->det_phase2++;
  int ok = 1;
  for (uint32_t w = 0; w < t->W; ++w) {
    uint64_t want_z = (w == (q >> 6)) ? (1ULL << (q & 63)) : 0;
    if (sx[w] != 0 || sz[w] != want_z) ok = 0;
  }
  if (!ok) t->badscratch++;
  free(sx); free(sz);
  *was_random = 0;
  return (int)sr;
}

/* Run a program of operations (type, q0, q1) in order. Gate runs are applied
 * to every held row; each OP_MEASURE takes the next measurement index m,
 * starting at meas_base, with coin(seed, shot, m). Outcome bytes and
 * was-random flags go to out_bits / out_random (either may be NULL), which
 * must hold one byte per measurement. Returns the number of measurements
 * completed: it stops early, before the first measurement the held rows cannot
 * decide. *ops_done receives the number of operations applied. */
int64_t sqo_run(sqo_tab *t, const uint32_t *ops, uint64_t count, uint64_t seed, uint64_t shot,
                uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random, uint64_t *ops_done) {
  uint64_t o = 0;
  int64_t m = 0;
  while (o < count) {
    if (ops[3 * o] != SQO_MEASURE) {
      uint64_t e = o;
      while (e < count && ops[3 * e] != SQO_MEASURE) ++e;
      apply_gate_run(t, ops + 3 * o, (size_t)(e - o));
      o = e;
      continue;
    }
    uint32_t q = ops[3 * o + 1];
    int coin = sqo_coin(seed, shot, meas_base + (uint64_t)m);
    int was_random = 0;
    int out = measure(t, q, coin, &was_random);
    if (out < 0) break;
    if (out_bits) out_bits[m] = (uint8_t)out;
    if (out_random) out_random[m] = (uint8_t)was_random;
    ++m;
    ++o;
  }
  if (ops_done) *ops_done = o;
  return m;
}

int sqo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Pauli-frame sampling ("Sampling" section, Algorithm alg:sampling), one
 * shot at a time. A shot's frame is a Pauli row (x and z bits over the n
 * qubits); gates conjugate it with the same rules as a tableau row (its sign
 * is not used). The frame starts with x = 0 and z drawn at random; measuring
 * qubit q records x_q and draws z_q afresh. The outcome of measurement i in
 * shot s is the reference sample's outcome i XOR the recorded x_q (the
 * paper records the frame bit alone; the reference XOR is the reading
 * taken here, which makes the outcome a sample of the circuit).
 *
 * Random bit of shot s for event e: bit (s mod 64) of output word 0 of
 * Philox4x64-10 with key (seed, 2^63 + floor(s / 64)) and counter
 * (e, 0, 0, 0); events 0..n-1 initialise z of each qubit, event n + i
 * re-draws z after measurement i. (The top key bit keeps these draws apart
 * from the measurement coins, keyed (seed, shot).)
 *
 * ops: count records (type, q0, q1) with type SQO_MEASURE for measurements;
 * ref: one byte per measurement; out: shots x W words, W = ceil(M / 64),
 * bit i of shot s at out[s * W + i / 64]. Returns M, or -1 on bad input. */
int sqo_frame_bit(uint64_t seed, uint64_t s, uint64_t e) {
  uint64_t ctr[4] = {e, 0, 0, 0}, key[2] = {seed, (1ULL << 63) + (s >> 6)}, out[4];
  sqo_philox4x64_10(ctr, key, out);
  return (int)((out[0] >> (s & 63)) & 1);
}

int64_t sqo_frame_sample(uint32_t n, const uint32_t *ops, uint64_t count, const uint8_t *ref, uint64_t seed,
                         uint32_t shots, uint64_t *out) {
  if (n == 0) return -1;
  uint64_t M = 0;
  for (uint64_t o = 0; o < count; ++o) {
    if (ops[3 * o] == SQO_MEASURE) ++M;
    if (ops[3 * o + 1] >= n) return -1;
  }
  const uint64_t W = (M + 63) / 64;
  const uint32_t nw = (n + 63) / 64;
  #pragma omp parallel for schedule(dynamic, 16)
  for (long s = 0; s < (long)shots; ++s) {
    uint64_t *x = (uint64_t *)calloc(nw, 8), *z = (uint64_t *)calloc(nw, 8);
    uint64_t *o_s = out + (size_t)s * W;
    for (uint64_t w = 0; w < W; ++w) o_s[w] = 0;
    for (uint32_t q = 0; q < n; ++q) putb(z, q, sqo_frame_bit(seed, (uint64_t)s, q));
    uint64_t i = 0;
    for (uint64_t o = 0; o < count; ++o) {
      const uint32_t t = ops[3 * o], a = ops[3 * o + 1], b = ops[3 * o + 2];
      if (t == SQO_MEASURE) {
        const int bit = (int)(ref[i] & 1) ^ getb(x, a);
        if (bit) o_s[i >> 6] |= 1ULL << (i & 63);
        putb(z, a, sqo_frame_bit(seed, (uint64_t)s, (uint64_t)n + i));
        ++i;
      } else {
        uint8_t sign = 0;
        gate_on_row(x, z, &sign, t, a, b);
      }
    }
    free(x);
    free(z);
  }
  return (int64_t)M;
}
