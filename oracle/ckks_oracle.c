/*
 * ckks_oracle.c -- CPU ORACLE, TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct modular arithmetic for the CKKS operations
 * behind HE-LRM's encrypted embedding lookup (paper Appendix A "CKKS
 * operations"; Sec. II-A "System-Level Costs" for key switching; Sec. II-A
 * "Neural Network Layers in FHE" for the diagonal matrix-vector method).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code with the GPU library: no
 * Shoup/Barrett/Montgomery tricks, every product is a full 128-bit integer
 * product followed by the C '%' operator.  Orchestration of the steps
 * (ModUp -> automorphism -> key inner product -> ModDown, the BSGS schedule,
 * rescale) lives in oracle.py, which calls these loops.
 *
 * Arrays of residues are laid out [limb][N] (limb-major, N contiguous words).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------ threads */

/* Thread count of the OpenMP loops below (the benchmark times the oracle
 * with one thread and with every host core). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------ scalars */

u64 or_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

u64 or_addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }

u64 or_submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - (b % q)) % q); }

u64 or_powmod(u64 a, u64 e, u64 q) {
  u64 r = 1 % q, b = a % q;
  while (e) {
    if (e & 1) r = or_mulmod(r, b, q);
    b = or_mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

/* Inverse modulo a prime by Fermat's little theorem. */
u64 or_invmod(u64 a, u64 q) { return or_powmod(a, q - 2, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases decide
 * primality for every n < 2^64 (Sorenson & Webster 2015). */
int or_is_prime(u64 n) {
  static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  u64 d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; r++; }
  for (int i = 0; i < 12; i++) {
    u64 x = or_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int k = 1; k < r; k++) {
      x = or_mulmod(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

/* The `count` largest primes q < bound with q = 1 (mod step), descending. */
int or_primes_below(u64 bound, u64 step, int count, u64 *out) {
  u64 k = (bound - 2) / step;
  int found = 0;
  while (found < count && k > 0) {
    u64 q = 1 + k * step;
    if (q < bound && or_is_prime(q)) out[found++] = q;
    k--;
  }
  return found;
}

/* psi = x^((q-1)/2N) for the smallest x >= 2 with x^((q-1)/2) = -1 (mod q).
 * Then psi^N = -1, so psi is a primitive 2N-th root of unity. */
u64 or_find_psi(u64 q, u64 N) {
  for (u64 x = 2;; x++) {
    if (or_powmod(x, (q - 1) / 2, q) == q - 1) return or_powmod(x, (q - 1) / (2 * N), q);
  }
}

static int ilog2(u64 n) { int l = 0; while ((1ULL << l) < n) l++; return l; }

u64 or_bitrev(u64 x, int bits) {
  u64 r = 0;
  for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* ------------------------------------------------------------ NTT */

/* Evaluation-form definition: out[j] = a(psi^(2*brv(j)+1)) mod q. O(N) per point. */
u64 or_ntt_definition_at(const u64 *a, int N, u64 q, u64 psi, int j) {
  int lg = ilog2((u64)N);
  u64 e = 2 * or_bitrev((u64)j, lg) + 1;
  u64 x = or_powmod(psi, e, q);
  /* Horner evaluation of a at x */
  u64 acc = 0;
  for (int c = N - 1; c >= 0; c--) acc = or_addmod(or_mulmod(acc, x, q), a[c] % q, q);
  return acc;
}

void or_ntt_definition(const u64 *a, u64 *out, int N, u64 q, u64 psi) {
  for (int j = 0; j < N; j++) out[j] = or_ntt_definition_at(a, N, q, psi, j);
}

/* Iterative radix-2 Cooley-Tukey transform whose output is the evaluation
 * form above (pinned against or_ntt_definition by the tests). In place. */
static void ntt_one(u64 *a, int N, u64 q, u64 psi) {
  int lg = ilog2((u64)N);
  u64 *pw = (u64 *)malloc(sizeof(u64) * N);
  pw[0] = 1;
  for (int k = 1; k < N; k++) pw[k] = or_mulmod(pw[k - 1], psi, q);
  for (int m = 1, len = N / 2; m < N; m <<= 1, len >>= 1) {
    for (int i = 0; i < m; i++) {
      u64 w = pw[or_bitrev((u64)(m + i), lg)];
      for (int j = 2 * i * len; j < 2 * i * len + len; j++) {
        u64 u = a[j], v = or_mulmod(a[j + len], w, q);
        a[j] = or_addmod(u, v, q);
        a[j + len] = or_submod(u, v, q);
      }
    }
  }
  free(pw);
}

/* Exact inverse of ntt_one: stages undone in reverse order, then times N^-1. */
static void intt_one(u64 *a, int N, u64 q, u64 psi) {
  int lg = ilog2((u64)N);
  u64 psi_inv = or_invmod(psi, q);
  u64 *pw = (u64 *)malloc(sizeof(u64) * N);
  pw[0] = 1;
  for (int k = 1; k < N; k++) pw[k] = or_mulmod(pw[k - 1], psi_inv, q);
  for (int m = N / 2, len = 1; m >= 1; m >>= 1, len <<= 1) {
    for (int i = 0; i < m; i++) {
      u64 w = pw[or_bitrev((u64)(m + i), lg)];
      for (int j = 2 * i * len; j < 2 * i * len + len; j++) {
        u64 u = a[j], v = a[j + len];
        a[j] = or_addmod(u, v, q);
        a[j + len] = or_mulmod(or_submod(u, v, q), w, q);
      }
    }
  }
  u64 ninv = or_invmod((u64)N % q, q);
  for (int j = 0; j < N; j++) a[j] = or_mulmod(a[j], ninv, q);
  free(pw);
}

void or_ntt(u64 *a, int nlimbs, int N, const u64 *q, const u64 *psi) {
#pragma omp parallel for schedule(dynamic)
  for (int l = 0; l < nlimbs; l++) ntt_one(a + (size_t)l * N, N, q[l], psi[l]);
}

void or_intt(u64 *a, int nlimbs, int N, const u64 *q, const u64 *psi) {
#pragma omp parallel for schedule(dynamic)
  for (int l = 0; l < nlimbs; l++) intt_one(a + (size_t)l * N, N, q[l], psi[l]);
}

/* Schoolbook product in Z_q[X]/(X^N+1): X^N = -1 folds the upper half back
 * with a minus sign. */
void or_negacyclic_schoolbook(const u64 *a, const u64 *b, u64 *out, int N, u64 q) {
  for (int k = 0; k < N; k++) out[k] = 0;
  for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
      u64 p = or_mulmod(a[i] % q, b[j] % q, q);
      int k = i + j;
      if (k < N) out[k] = or_addmod(out[k], p, q);
      else out[k - N] = or_submod(out[k - N], p, q);
    }
}

/* ------------------------------------------------------------ automorphism */

/* Coefficient form: sigma_g(a)(X) = a(X^g).  X^c -> X^(c*g mod 2N), and an
 * exponent e >= N lands on X^(e-N) with a minus sign (X^N = -1). */
void or_automorph_coeff(const u64 *in, u64 *out, int nlimbs, int N, const u64 *q, u64 g) {
  for (int l = 0; l < nlimbs; l++) {
    const u64 *a = in + (size_t)l * N;
    u64 *o = out + (size_t)l * N;
    for (int c = 0; c < N; c++) {
      u64 e = ((u128)c * g) % (u64)(2 * N);
      if (e < (u64)N) o[e] = a[c] % q[l];
      else o[e - N] = or_submod(0, a[c], q[l]);
    }
  }
}

/* Evaluation form: sigma_g(a) evaluated at psi^(2 brv(j)+1) equals a evaluated
 * at psi^(g (2 brv(j)+1)); that point is index j' with 2 brv(j')+1 = g(2 brv(j)+1). */
void or_automorph_ntt(const u64 *in, u64 *out, int nlimbs, int N, u64 g) {
  int lg = ilog2((u64)N);
  for (int j = 0; j < N; j++) {
    u64 e = 2 * or_bitrev((u64)j, lg) + 1;
    u64 e2 = ((u128)e * g) % (u64)(2 * N);
    u64 jp = or_bitrev((e2 - 1) / 2, lg);
    for (int l = 0; l < nlimbs; l++) out[(size_t)l * N + j] = in[(size_t)l * N + jp];
  }
}

/* ------------------------------------------------------------ elementwise */

void or_mul(const u64 *a, const u64 *b, u64 *out, int nlimbs, int N, const u64 *q) {
#pragma omp parallel for
  for (int l = 0; l < nlimbs; l++)
    for (int j = 0; j < N; j++) {
      size_t x = (size_t)l * N + j;
      out[x] = or_mulmod(a[x], b[x], q[l]);
    }
}

void or_add(const u64 *a, const u64 *b, u64 *out, int nlimbs, int N, const u64 *q) {
#pragma omp parallel for
  for (int l = 0; l < nlimbs; l++)
    for (int j = 0; j < N; j++) {
      size_t x = (size_t)l * N + j;
      out[x] = or_addmod(a[x], b[x], q[l]);
    }
}

void or_sub(const u64 *a, const u64 *b, u64 *out, int nlimbs, int N, const u64 *q) {
#pragma omp parallel for
  for (int l = 0; l < nlimbs; l++)
    for (int j = 0; j < N; j++) {
      size_t x = (size_t)l * N + j;
      out[x] = or_submod(a[x], b[x], q[l]);
    }
}

/* out[l][j] = a[l][j] * s[l] mod q[l] (one scalar per limb). */
void or_mul_scalar(const u64 *a, const u64 *s, u64 *out, int nlimbs, int N, const u64 *q) {
#pragma omp parallel for
  for (int l = 0; l < nlimbs; l++)
    for (int j = 0; j < N; j++) {
      size_t x = (size_t)l * N + j;
      out[x] = or_mulmod(a[x], s[l] % q[l], q[l]);
    }
}

/* Signed integers to residues: out[l][j] = v[j] mod q[l] in [0, q[l]). */
void or_from_signed(const int64_t *v, u64 *out, int nlimbs, int N, const u64 *q) {
  for (int l = 0; l < nlimbs; l++)
    for (int j = 0; j < N; j++) {
      int64_t x = v[j];
      u64 r = (x >= 0) ? ((u64)x % q[l]) : or_submod(0, ((u64)(-(x + 1)) + 1) % q[l], q[l]);
      out[(size_t)l * N + j] = r;
    }
}

/* ------------------------------------------------------------ basis conversion */

/* Fast base conversion of coefficient-form residues x over the input primes
 * qin[0..nin) to the output primes qout[0..nout):
 *   y_i  = x_i * (Qin/qin_i)^-1 mod qin_i
 *   out_r = sum_i y_i * (Qin/qin_i mod r) mod r.
 * The integer sum_i y_i (Qin/qin_i) equals [x]_Qin + u Qin with 0 <= u < nin. */
void or_basis_convert(const u64 *x, int nin, const u64 *qin, u64 *out, int nout,
                      const u64 *qout, int N) {
  u64 *hat_inv = (u64 *)malloc(sizeof(u64) * nin);
  u64 *hat_out = (u64 *)malloc(sizeof(u64) * nin * nout);
  for (int i = 0; i < nin; i++) {
    u64 h = 1; /* Qin/qin_i mod qin_i */
    for (int k = 0; k < nin; k++) if (k != i) h = or_mulmod(h, qin[k] % qin[i], qin[i]);
    hat_inv[i] = or_invmod(h, qin[i]);
    for (int r = 0; r < nout; r++) {
      u64 hr = 1; /* Qin/qin_i mod qout_r */
      for (int k = 0; k < nin; k++) if (k != i) hr = or_mulmod(hr, qin[k] % qout[r], qout[r]);
      hat_out[i * nout + r] = hr;
    }
  }
#pragma omp parallel for
  for (int j = 0; j < N; j++) {
    u64 y[64];
    for (int i = 0; i < nin; i++) y[i] = or_mulmod(x[(size_t)i * N + j], hat_inv[i], qin[i]);
    for (int r = 0; r < nout; r++) {
      u64 acc = 0;
      for (int i = 0; i < nin; i++)
        acc = or_addmod(acc, or_mulmod(y[i] % qout[r], hat_out[i * nout + r], qout[r]), qout[r]);
      out[(size_t)r * N + j] = acc;
    }
  }
  free(hat_inv);
  free(hat_out);
}

/* ------------------------------------------------------------ seeded uniform key polynomials
 *
 * The uniform part a_j of a switching key is expanded from the key's 64-bit
 * seed with SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014): output n >= 1 of the generator seeded with
 * s is mix(s + n * 0x9E3779B97F4A7C15), where mix is the finaliser below.
 * Value x of digit j on prime index p is drawn from counter c = x + 2^16 p +
 * 2^24 j.  On a prime of 40 bits or more it is the 128-bit integer
 * X = out_{2c+2} 2^64 + out_{2c+1}, whose residue mod q is within q / 2^128
 * < 2^-68 of uniform.  On a prime below 2^40 it is one 64-bit output taken by
 * rejection: candidate 0 is out_{2c+1}, candidate t = 1, 2, 3 is
 * out_{2^32 + 4c + t} (a range no other counter reaches); the first candidate
 * below lambda = 2^64 - (2^64 mod q), the largest multiple of q not above
 * 2^64, is X (candidate 3 if none is), so X mod q is uniform on [0, q) up to
 * the chance 2^-96 that all four are rejected.  The key value is
 * a = (X mod q) * 2^-128 mod q: a fixed bijection of X mod q, so exactly as
 * uniform, chosen so that its Montgomery-form value (X mod q) * 2^-64 is one
 * reduction of X. */

u64 or_splitmix64(u64 seed, u64 n) {
  u64 z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The 64-bit sample of counter c on a prime below 2^40 (rejection, above). */
u64 or_key_uniform_sample40(u64 seed, u64 c, u64 q) {
  const u64 lambda = (u64)0 - (u64)(((u128)1 << 64) % q);   /* 2^64 - (2^64 mod q) */
  u64 X = or_splitmix64(seed, 2 * c + 1);
  for (u64 t = 1; t <= 3 && X >= lambda; t++) X = or_splitmix64(seed, ((u64)1 << 32) + 4 * c + t);
  return X;
}

void or_key_uniform(u64 seed, int j, int p, u64 q, int N, u64 *out) {
  /* 2^-128 mod q */
  const u64 two64 = (u64)(((u128)1 << 64) % q);
  const u64 inv128 = or_invmod(or_mulmod(two64, two64, q), q);
  for (int x = 0; x < N; x++) {
    const u64 c = (u64)x + ((u64)p << 16) + ((u64)j << 24);
    u128 X;
    if (q < ((u64)1 << 40))
      X = or_key_uniform_sample40(seed, c, q);
    else
      X = ((u128)or_splitmix64(seed, 2 * c + 2) << 64) | or_splitmix64(seed, 2 * c + 1);
    out[x] = or_mulmod((u64)(X % q), inv128, q);
  }
}
