/*
 * CPU oracle of the paper's own measurement procedure, the CX-injection
 * collapse of Algorithm alg:stim -- TEST INFRASTRUCTURE ONLY.
 *
 * The collapse works on the operator tableau T = C^dagger of the circuit C
 * that prepared the state C|0...0>: for each qubit q the two Pauli strings
 * A_q = T(X_q) and B_q = T(Z_q) over the generator positions k = 0..n-1,
 * each with a sign. The paper writes its bits as four n x n matrices indexed
 * [generator k, qubit q] (Algorithm alg:stim, bracket notation):
 *   XS[k][q] = x bit of B_q at k,   XD[k][q] = z bit of B_q at k,
 *   ZS[k][q] = x bit of A_q at k,   ZD[k][q] = z bit of A_q at k,
 * and two sign vectors indexed by qubit: SignsS[q] = sign of B_q,
 * SignsD[q] = sign of A_q. (These four matrices hold exactly the bits of
 * the CHP state tableau, XS[k][q] = x_q(S_k), XD[k][q] = x_q(D_k) and so
 * on; only the signs are indexed differently.) Row k of a matrix is stored
 * as W = ceil(n/64) words over q, LSB first.
 *
 * Gates act on the strings of their qubits: applying U after C gives
 * T'(P) = T(U^dagger P U), e.g. H exchanges A_q and B_q, S makes A_q the
 * product -i A_q B_q, CX(c, t) makes A_c = A_c A_t and B_t = B_c B_t; products
 * carry the phase of the Aaronson-Gottesman g function.
 *
 * Measuring Z_q follows Algorithm alg:stim step by step: the pivot p is the
 * smallest k with XS[k][q] = 1; if there is one, every later generator t
 * with XS[t][q] = 1 gets a CX injected from p (the CX conjugation rule on
 * the pair of positions (p, t), applied to every string: InjectCX on
 * (SignsD, ZS[p], ZD[p], ZS[t], ZD[t]) and on (SignsS, XS[p], XD[p], XS[t],
 * XD[t]) with the whole rows as operands), then the pivot position is rotated
 * so that B_q has no x bit left (H_YZ, the paper's InjectInvP, when
 * XD[p][q] = 1, else H), and when SignsS[q] differs from the coin an X is
 * injected at p (the signs take the z bits of row p). The outcome is
 * SignsS[q], in both the random and the deterministic case. Coins are those
 * of the CHP oracle (sqo_coin), so both give the same outcomes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int sqo_coin(uint64_t seed, uint64_t shot, uint64_t m);
int sqo_g(int x1, int z1, int x2, int z2);

enum {
  OT_H = 1, OT_S = 2, OT_SDG = 3, OT_X = 4, OT_Y = 5, OT_Z = 6,
  OT_CX = 7, OT_CZ = 8, OT_CY = 9, OT_SWAP = 10, OT_ISWAP = 11, OT_MEASURE = 15
};

typedef struct {
  uint32_t n, W;
  uint64_t *xs, *xd, *zs, *zd;  /* n rows (generator k) of W words (qubits) */
  uint64_t *ss, *sd;            /* W words: SignsS[q], SignsD[q] */
  uint64_t odd;                 /* products whose phase was not real (must stay 0) */
} sqo_otab;

static inline int bit(const uint64_t *v, uint32_t j) { return (int)((v[j >> 6] >> (j & 63)) & 1); }
static inline void setbit(uint64_t *v, uint32_t j, int b) {
  const uint64_t m = 1ULL << (j & 63);
  if (b) v[j >> 6] |= m; else v[j >> 6] &= ~m;
}

sqo_otab *sqo_otab_create(uint32_t n) {
  if (n == 0) return NULL;
  sqo_otab *t = (sqo_otab *)calloc(1, sizeof(sqo_otab));
  t->n = n;
  t->W = (n + 63) / 64;
  const size_t words = (size_t)n * t->W;
  t->xs = (uint64_t *)calloc(words, 8);
  t->xd = (uint64_t *)calloc(words, 8);
  t->zs = (uint64_t *)calloc(words, 8);
  t->zd = (uint64_t *)calloc(words, 8);
  t->ss = (uint64_t *)calloc(t->W, 8);
  t->sd = (uint64_t *)calloc(t->W, 8);
  /* |0...0>: C = I, so A_q = X_q (ZS = I) and B_q = Z_q (XD = I) */
  for (uint32_t k = 0; k < n; ++k) {
    setbit(t->zs + (size_t)k * t->W, k, 1);
    setbit(t->xd + (size_t)k * t->W, k, 1);
  }
  return t;
}

void sqo_otab_destroy(sqo_otab *t) {
  if (!t) return;
  free(t->xs); free(t->xd); free(t->zs); free(t->zd); free(t->ss); free(t->sd);
  free(t);
}

uint64_t sqo_otab_odd_count(const sqo_otab *t) { return t->odd; }

/* The string of qubit q: A_q (which = 0) or B_q (which = 1). */
typedef struct { uint64_t *x, *z, *s; uint32_t q; } ostr;
static ostr str_of(sqo_otab *t, uint32_t q, int which) {
  ostr r;
  r.x = which ? t->xs : t->zs;
  r.z = which ? t->xd : t->zd;
  r.s = which ? t->ss : t->sd;
  r.q = q;
  return r;
}

/* P <- i^extra * P * Q (P first), over the n positions; the phase exponent
 * 2 s_P + 2 s_Q + extra + sum_k g(P_k, Q_k) must be even. */
static void str_mul(sqo_otab *t, ostr P, ostr Q, int extra) {
  const uint32_t n = t->n, W = t->W;
  int e = 2 * bit(P.s, P.q) + 2 * bit(Q.s, Q.q) + extra;
  for (uint32_t k = 0; k < n; ++k) {
    const size_t o = (size_t)k * W;
    const int px = bit(P.x + o, P.q), pz = bit(P.z + o, P.q);
    const int qx = bit(Q.x + o, Q.q), qz = bit(Q.z + o, Q.q);
    e += sqo_g(px, pz, qx, qz);
    setbit(P.x + o, P.q, px ^ qx);
    setbit(P.z + o, P.q, pz ^ qz);
  }
  e = ((e % 4) + 4) % 4;
  if (e & 1) t->odd++;
  setbit(P.s, P.q, e >> 1);
}

static void str_swap(sqo_otab *t, ostr P, ostr Q) {
  const uint32_t n = t->n, W = t->W;
  for (uint32_t k = 0; k < n; ++k) {
    const size_t o = (size_t)k * W;
    const int px = bit(P.x + o, P.q), pz = bit(P.z + o, P.q);
    setbit(P.x + o, P.q, bit(Q.x + o, Q.q));
    setbit(P.z + o, P.q, bit(Q.z + o, Q.q));
    setbit(Q.x + o, Q.q, px);
    setbit(Q.z + o, Q.q, pz);
  }
  const int ps = bit(P.s, P.q);
  setbit(P.s, P.q, bit(Q.s, Q.q));
  setbit(Q.s, Q.q, ps);
}

static void flip_sign(ostr P) { setbit(P.s, P.q, bit(P.s, P.q) ^ 1); }

/* Apply one gate after the circuit: T'(P) = T(U^dagger P U) on the strings
 * of its qubits. S^dagger X S = -Y = -i X Z, S X S^dagger = Y = i X Z;
 * CX maps X_c to X_c X_t and Z_t to Z_c Z_t; CZ maps X_a to X_a Z_b; X, Z, Y
 * negate the images of the Paulis they anticommute with. CY and iSWAP are
 * taken as the same products, in the same time order, as the CHP oracle's. */
static void otab_gate(sqo_otab *t, uint32_t type, uint32_t a, uint32_t b) {
  switch (type) {
    case OT_H: str_swap(t, str_of(t, a, 0), str_of(t, a, 1)); break;
    case OT_S: str_mul(t, str_of(t, a, 0), str_of(t, a, 1), 3); break;    /* A <- -i A B */
    case OT_SDG: str_mul(t, str_of(t, a, 0), str_of(t, a, 1), 1); break;  /* A <- i A B */
    case OT_X: flip_sign(str_of(t, a, 1)); break;
    case OT_Z: flip_sign(str_of(t, a, 0)); break;
    case OT_Y: flip_sign(str_of(t, a, 0)); flip_sign(str_of(t, a, 1)); break;
    case OT_CX:
      str_mul(t, str_of(t, a, 0), str_of(t, b, 0), 0);  /* A_c <- A_c A_t */
      str_mul(t, str_of(t, b, 1), str_of(t, a, 1), 0);  /* B_t <- B_t B_c (they commute) */
      break;
    case OT_CZ:
      str_mul(t, str_of(t, a, 0), str_of(t, b, 1), 0);  /* A_a <- A_a B_b */
      str_mul(t, str_of(t, b, 0), str_of(t, a, 1), 0);  /* A_b <- A_b B_a */
      break;
    case OT_SWAP:
      str_swap(t, str_of(t, a, 0), str_of(t, b, 0));
      str_swap(t, str_of(t, a, 1), str_of(t, b, 1));
      break;
    case OT_CY:
      otab_gate(t, OT_SDG, b, 0);
      otab_gate(t, OT_CX, a, b);
      otab_gate(t, OT_S, b, 0);
      break;
    case OT_ISWAP:
      otab_gate(t, OT_S, a, 0);
      otab_gate(t, OT_S, b, 0);
      otab_gate(t, OT_CZ, a, b);
      otab_gate(t, OT_SWAP, a, b);
      break;
    default:
      break;
  }
}

/* The four word-vector updates of Algorithm alg:stim, over whole rows. */
static void inject_cx(uint64_t *s, const uint64_t *xc, uint64_t *zc, uint64_t *xt, const uint64_t *zt, uint32_t W) {
  for (uint32_t w = 0; w < W; ++w) {
    s[w] ^= xc[w] & zt[w] & ~(zc[w] ^ xt[w]);
    xt[w] ^= xc[w];
    zc[w] ^= zt[w];
  }
}

static void inject_invp(uint64_t *s, uint64_t *x, const uint64_t *z, uint32_t W) {
  for (uint32_t w = 0; w < W; ++w) {
    s[w] ^= x[w] & ~z[w];
    x[w] ^= z[w];
  }
}

static void inject_had(uint64_t *s, uint64_t *x, uint64_t *z, uint32_t W) {
  for (uint32_t w = 0; w < W; ++w) {
    s[w] ^= x[w] & z[w];
    const uint64_t tmp = x[w];
    x[w] = z[w];
    z[w] = tmp;
  }
}

static void inject_x(uint64_t *s, const uint64_t *z, uint32_t W) {
  for (uint32_t w = 0; w < W; ++w) s[w] ^= z[w];
}

/* Measure Z_q with the given coin (Algorithm alg:stim); returns the outcome. */
static int otab_measure(sqo_otab *t, uint32_t q, int coin, int *was_random) {
  const uint32_t n = t->n, W = t->W;
  int32_t p = -1;
  for (uint32_t k = 0; k < n; ++k)
    if (bit(t->xs + (size_t)k * W, q)) { p = (int32_t)k; break; }
  *was_random = p >= 0;
  if (p >= 0) {
    uint64_t *xsp = t->xs + (size_t)p * W, *xdp = t->xd + (size_t)p * W;
    uint64_t *zsp = t->zs + (size_t)p * W, *zdp = t->zd + (size_t)p * W;
    /* Gaussian elimination: targets in strictly increasing order */
    for (uint32_t k = (uint32_t)p + 1; k < n; ++k) {
      if (!bit(t->xs + (size_t)k * W, q)) continue;
      inject_cx(t->sd, zsp, zdp, t->zs + (size_t)k * W, t->zd + (size_t)k * W, W);
      inject_cx(t->ss, xsp, xdp, t->xs + (size_t)k * W, t->xd + (size_t)k * W, W);
    }
    /* swap the anticommuting generator for one that commutes with Z_q */
    if (bit(xdp, q)) {
      inject_invp(t->sd, zsp, zdp, W);
      inject_invp(t->ss, xsp, xdp, W);
    } else {
      inject_had(t->sd, zsp, zdp, W);
      inject_had(t->ss, xsp, xdp, W);
    }
    if (bit(t->ss, q) != coin) {
      inject_x(t->sd, zdp, W);
      inject_x(t->ss, xdp, W);
    }
  }
  return bit(t->ss, q);
}

/* Run operations (type, q0, q1) in order; measurement m (from meas_base)
 * draws sqo_coin(seed, shot, m). Writes outcomes and was-random flags (either
 * may be NULL) and returns the number of measurements. */
int64_t sqo_otab_run(sqo_otab *t, const uint32_t *ops, uint64_t count, uint64_t seed, uint64_t shot,
                     uint64_t meas_base, uint8_t *out_bits, uint8_t *out_random) {
  int64_t m = 0;
  for (uint64_t o = 0; o < count; ++o) {
    const uint32_t type = ops[3 * o], a = ops[3 * o + 1], b = ops[3 * o + 2];
    if (type != OT_MEASURE) {
      otab_gate(t, type, a, b);
      continue;
    }
    int rnd = 0;
    const int out = otab_measure(t, a, sqo_coin(seed, shot, meas_base + (uint64_t)m), &rnd);
    if (out_bits) out_bits[m] = (uint8_t)out;
    if (out_random) out_random[m] = (uint8_t)rnd;
    ++m;
  }
  return m;
}

/* Copy the matrices (n x W words each, row k = generator k) and sign vectors
 * (W words each) out or in. */
void sqo_otab_get(const sqo_otab *t, uint64_t *xs, uint64_t *xd, uint64_t *zs, uint64_t *zd, uint64_t *ss,
                  uint64_t *sd) {
  const size_t words = (size_t)t->n * t->W;
  memcpy(xs, t->xs, words * 8);
  memcpy(xd, t->xd, words * 8);
  memcpy(zs, t->zs, words * 8);
  memcpy(zd, t->zd, words * 8);
  memcpy(ss, t->ss, (size_t)t->W * 8);
  memcpy(sd, t->sd, (size_t)t->W * 8);
}

void sqo_otab_set(sqo_otab *t, const uint64_t *xs, const uint64_t *xd, const uint64_t *zs, const uint64_t *zd,
                  const uint64_t *ss, const uint64_t *sd) {
  const size_t words = (size_t)t->n * t->W;
  memcpy(t->xs, xs, words * 8);
  memcpy(t->xd, xd, words * 8);
  memcpy(t->zs, zs, words * 8);
  memcpy(t->zd, zd, words * 8);
  memcpy(t->ss, ss, (size_t)t->W * 8);
  memcpy(t->sd, sd, (size_t)t->W * 8);
}

/* The image T(P) of a Pauli P = (-1)^r P_0 ... P_{n-1} given in the CHP
 * encoding (x, z: W words over qubits; P_q = X, Z, Y for (1,0), (0,1),
 * (1,1), with Y = i X Z): T(P) = (-1)^r prod_q T(P_q), taken qubit by qubit.
 * Writes its bits over the generator positions (ox, oz: W words) and sign;
 * returns 1 if the product's phase was not real. */
int sqo_otab_image(sqo_otab *t, const uint64_t *x, const uint64_t *z, int r, uint64_t *ox, uint64_t *oz,
                   uint8_t *osign) {
  const uint32_t n = t->n, W = t->W;
  memset(ox, 0, (size_t)W * 8);
  memset(oz, 0, (size_t)W * 8);
  int e = 2 * (r & 1);  /* exponent of i */
  for (uint32_t q = 0; q < n; ++q) {
    const int xq = bit(x, q), zq = bit(z, q);
    if (!xq && !zq) continue;
    if (xq && zq) e += 1;  /* Y = i X Z */
    for (int which = 0; which < 2; ++which) {
      if (which == 0 && !xq) continue;
      if (which == 1 && !zq) continue;
      ostr F = str_of(t, q, which);
      e += 2 * bit(F.s, q);
      for (uint32_t k = 0; k < n; ++k) {
        const size_t o = (size_t)k * W;
        const int fx = bit(F.x + o, q), fz = bit(F.z + o, q);
        e += sqo_g(bit(ox, k), bit(oz, k), fx, fz);
        setbit(ox, k, bit(ox, k) ^ fx);
        setbit(oz, k, bit(oz, k) ^ fz);
      }
    }
  }
  e = ((e % 4) + 4) % 4;
  *osign = (uint8_t)(e >> 1);
  return e & 1;
}
