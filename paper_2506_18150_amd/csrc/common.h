// Internal declarations of libhelrm: device modular arithmetic, launch
// descriptors, the context structure and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "helrm.h"

typedef uint64_t u64;
typedef unsigned __int128 u128;

#define HELRM_MAX_PRIMES 64   // L+1+K
#define HELRM_MAX_LIMBS 128   // limbs one descriptor list may name
#define HELRM_MAX_TERMS 16    // key-switch terms summed by one accumulate launch
#define HELRM_MAX_BABY 64     // baby steps per fused MAC launch
#define HELRM_MAX_GTILE 8     // giant outputs accumulated per fused MAC launch
#define HELRM_MAX_CONV_JOBS 4 // base conversions per launch

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
      return HELRM_EHIP;                                                           \
    }                                                                              \
  } while (0)

#define CHECK_ARG(cond, ...)          \
  do {                                \
    if (!(cond)) {                    \
      set_error(__VA_ARGS__);         \
      return HELRM_EINVAL;            \
    }                                 \
  } while (0)

#define TRY(expr)                     \
  do {                                \
    int _r = (expr);                  \
    if (_r != HELRM_OK) return _r;    \
  } while (0)

// ---------------------------------------------------------------- device arithmetic
//
// Two reductions are used:
//  * Shoup: x * w mod q for a fixed w with w' = floor(w 2^64 / q); the result
//    of the lazy form is in [0, 2q) for any 64-bit x (Shoup; Harvey 2014).
//  * Montgomery REDC (Montgomery 1985): for T = hi 2^64 + lo with hi < q,
//    returns T 2^-64 mod q.  Resident operands (keys, plaintext diagonals,
//    conversion constants) are stored pre-multiplied by 2^64, so REDC of a
//    128-bit sum of products gives the plain modular sum of products.

struct Mod {
  u64 q;
  u64 qn;  // -q^-1 mod 2^64
};

__device__ __forceinline__ u64 shoup_lazy(u64 x, u64 w, u64 wp, u64 q) {
  u64 qh = __umul64hi(x, wp);
  return x * w - qh * q;
}

__device__ __forceinline__ u64 shoup(u64 x, u64 w, u64 wp, u64 q) {
  u64 r = shoup_lazy(x, w, wp, q);
  return r >= q ? r - q : r;
}

struct Acc {
  u64 lo, hi;
};

__device__ __forceinline__ void acc_zero(Acc &a) { a.lo = 0; a.hi = 0; }

__device__ __forceinline__ void acc_mac(Acc &a, u64 x, u64 y) {
  u128 p = (u128)x * y;
  u64 l = (u64)p;
  a.lo += l;
  a.hi += (u64)(p >> 64) + (a.lo < l ? 1 : 0);
}

// REDC for hi < q: result in [0, q).
__device__ __forceinline__ u64 redc(u64 lo, u64 hi, u64 q, u64 qn) {
  u64 m = lo * qn;
  u64 r = hi + __umul64hi(m, q) + (lo != 0 ? 1 : 0);
  return r >= q ? r - q : r;
}

// REDC for hi < 4q (sums of up to 64 products of residues below 2^60).
__device__ __forceinline__ u64 redc_acc(const Acc &a, u64 q, u64 qn) {
  u64 hi = a.hi;
  hi = hi >= 2 * q ? hi - 2 * q : hi;
  hi = hi >= q ? hi - q : hi;
  return redc(a.lo, hi, q, qn);
}

// Multiply-accumulate policies for sums of at most 64 products of residues,
// finished by one REDC.  Both give the same canonical result, REDC(exact sum).
//
// WideMac: 128-bit lazy sum, any residue below 2^60.
struct WideMac {
  using Op = u64;
  Acc a;
  static __device__ __forceinline__ Op prep(u64 v) { return v; }
  __device__ __forceinline__ void zero() { acc_zero(a); }
  __device__ __forceinline__ void mac(Op x, Op y) { acc_mac(a, x, y); }
  __device__ __forceinline__ u64 finish(u64 q, u64 qn) const { return redc_acc(a, q, qn); }
};

// SplitMac: residues below 2^40 split into 20-bit halves x = x0 + 2^20 x1;
// x y = x0 y0 + 2^20 ((x0+x1)(y0+y1) - x0 y0 - x1 y1) + 2^40 x1 y1 (Karatsuba),
// so a product costs three 32x32->64 multiply-adds into three 64-bit sums
// that cannot overflow (64 products: below 2^46, 2^46, 2^48).  The exact sum
// (below 2^86, so its high word is below q) is rebuilt once, then REDC.
struct Half20 {
  uint32_t lo, hi, sum;
};
struct SplitMac {
  using Op = Half20;
  u64 s0, s1, sm;
  static __device__ __forceinline__ Op prep(u64 v) {
    Half20 h;
    h.lo = (uint32_t)v & 0xFFFFFu;
    h.hi = (uint32_t)(v >> 20);
    h.sum = h.lo + h.hi;
    return h;
  }
  __device__ __forceinline__ void zero() { s0 = s1 = sm = 0; }
  __device__ __forceinline__ void mac(const Op &x, const Op &y) {
    s0 += (u64)x.lo * y.lo;
    s1 += (u64)x.hi * y.hi;
    sm += (u64)x.sum * y.sum;
  }
  __device__ __forceinline__ u64 finish(u64 q, u64 qn) const {
    const u64 mid = sm - s0 - s1;
    u128 s = (u128)s0 + ((u128)mid << 20) + ((u128)s1 << 40);
    return redc((u64)s, (u64)(s >> 64), q, qn);
  }
};

constexpr u64 SPLIT_MAC_LIMIT = 1ull << 40;   // SplitMac needs every residue below this

// Sum of at most 16 products of residues below 2^60 in 30-bit halves:
// x = x0 + 2^30 x1, y = y0 + 2^30 y1, so x y = x0 y0 + 2^30 (x0 y1 + x1 y0)
// + 2^60 x1 y1.  Each half-product is one 32x32->64 multiply-add and below
// 2^60, so the four 64-bit partial sums cannot overflow for 16 terms; the
// exact sum (the same value a 128-bit accumulator holds) is rebuilt once.
// Operands are packed as lo | hi << 32.
__device__ __forceinline__ u64 split30(u64 v) { return (v & 0x3FFFFFFFull) | ((v >> 30) << 32); }

struct Sum30 {
  u64 s00, s01, s10, s11;
  __device__ __forceinline__ void zero() { s00 = s01 = s10 = s11 = 0; }
  __device__ __forceinline__ void mac(u64 x, u64 y) {   // both split30-packed
    const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32), y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
    s00 += (u64)x0 * y0;
    s01 += (u64)x0 * y1;
    s10 += (u64)x1 * y0;
    s11 += (u64)x1 * y1;
  }
  __device__ __forceinline__ Acc value() const {
    const u128 v = (u128)s00 + ((u128)s01 << 30) + ((u128)s10 << 30) + ((u128)s11 << 60);
    return Acc{(u64)v, (u64)(v >> 64)};
  }
};

// Wide30Mac: WideMac's result for residues below 2^60 at four 32-bit
// multiply-adds per product: products go into a Sum30, which is folded into
// the 128-bit total every 16 products (and at the end).  Twelve registers per
// accumulator, so kernels use it where a thread holds few accumulators.
struct Wide30Mac {
  using Op = u64;   // split30-packed
  Sum30 s;
  Acc a;
  int n;
  static __device__ __forceinline__ Op prep(u64 v) { return split30(v); }
  __device__ __forceinline__ void zero() {
    s.zero();
    acc_zero(a);
    n = 0;
  }
  __device__ __forceinline__ void fold() {
    const Acc v = s.value();
    a.lo += v.lo;
    a.hi += v.hi + (a.lo < v.lo ? 1 : 0);
    s.zero();
    n = 0;
  }
  __device__ __forceinline__ void mac(Op x, Op y) {
    s.mac(x, y);
    if (++n == 16) fold();
  }
  __device__ __forceinline__ u64 finish(u64 q, u64 qn) const {
    const Acc v = s.value();
    Acc t = a;
    t.lo += v.lo;
    t.hi += v.hi + (t.lo < v.lo ? 1 : 0);
    return redc_acc(t, q, qn);
  }
};

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}

__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) {
  return a >= b ? a - b : a + q - b;
}

// x mod q for any 64-bit x, with mu = floor(2^64 / q).
__device__ __forceinline__ u64 reduce64(u64 x, u64 q, u64 mu) {
  u64 r = x - __umul64hi(x, mu) * q;
  return r >= q ? r - q : r;
}

// Evaluation-form index permutation of X -> X^g:
// out[j] = in[j'] with 2 brv(j')+1 = g (2 brv(j)+1) mod 2N.
__device__ __forceinline__ unsigned galois_src(unsigned j, unsigned g, int logn) {
  unsigned e = 2u * (__brev(j) >> (32 - logn)) + 1u;
  unsigned e2 = (g * e) & ((2u << logn) - 1u);
  return __brev((e2 - 1u) >> 1) >> (32 - logn);
}

// Uniform half a_j of a switching key, regenerated from the key's seed with
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output n of the generator
// seeded with s is mix(s + n * 0x9E3779B97F4A7C15).  Value x of digit j on
// prime index p draws from counter c = x + 2^16 p + 2^24 j: on primes of 40
// bits or more X = out_{2c+2} 2^64 + out_{2c+1} (within 2^-68 of uniform mod
// q); below 2^40 X is the first of out_{2c+1}, out_{2^32+4c+t} (t = 1..3)
// below 2^64 - (2^64 mod q) (rejection: X mod q exactly uniform but for a
// 2^-96 tail).  The key holds a_j = (X mod q) 2^-128, whose Montgomery form
// is X 2^-64 mod q = REDC((out_{2c+2} mod q) 2^64 + out_{2c+1}), or REDC(X)
// for the 64-bit X.
constexpr u64 SM_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ u64 sm_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- per-prime device constants

struct PrimeInfo {
  u64 q, qn;           // modulus, -q^-1 mod 2^64
  u64 mu;              // floor(2^64 / q)
  u64 r2;              // 2^128 mod q (to Montgomery form: REDC(x r2) = x 2^64)
  u64 ninv, ninv_p;    // N^-1 mod q with its Shoup companion
  u64 pmod, pmod_p;    // [P]_q with Shoup companion (P = product of special primes)
  u64 pinv, pinv_p;    // [P^-1]_q (Q primes only)
  double qd, qinv_d;   // q and 1/q as doubles (fp64 NTT path, q < 2^41)
  double ninv_d;       // N^-1 mod q as a double
  u64 lam;             // 2^64 - (2^64 mod q): 64-bit key samples at or above it are rejected
};

struct TW {
  u64 w, wp;
};

// Montgomery-form a_j value of a seeded key at (digit j, prime index p,
// coefficient x).  A rejected first candidate (probability below 2^-24 per
// word) sends the lane through the retry loop.
__device__ __forceinline__ u64 key_uniform_mont(u64 seed, int j, int p, int x, const PrimeInfo &pi) {
  const u64 c = (u64)x + ((u64)p << 16) + ((u64)j << 24);
  u64 lo = sm_mix(seed + (2 * c + 1) * SM_GAMMA);
  if (pi.q < SPLIT_MAC_LIMIT) {
    if (lo >= pi.lam) {
#pragma unroll 1
      for (u64 t = 1; t <= 3; t++) {
        lo = sm_mix(seed + ((1ull << 32) + 4 * c + t) * SM_GAMMA);
        if (lo < pi.lam) break;
      }
    }
    return redc(lo, 0, pi.q, pi.qn);
  }
  const u64 hi = sm_mix(seed + (2 * c + 2) * SM_GAMMA);
  return redc(lo, reduce64(hi, pi.q, pi.mu), pi.q, pi.qn);
}

// A list of limbs for one launch.  Limb i of batch element b lives at
// base + (b * bstride + off[i]) * N and uses prime prime[i].
struct LimbList {
  int n;
  int src_bstride;   // in limbs
  int dst_bstride;   // in limbs
  int src_off[HELRM_MAX_LIMBS];
  int dst_off[HELRM_MAX_LIMBS];
  int prime[HELRM_MAX_LIMBS];        // int, not byte: a uniform index reads it with a scalar load
};

// Fast base conversion for one (level, digit) or the ModDown of one level.
struct ConvTable {
  int nin, nout;
  int in_prime[16];
  int out_prime[HELRM_MAX_PRIMES];
  // device pointers into the context's constant buffer
  const TW *hat_inv;   // [nin]: (Qin/q_i)^-1 mod q_i, Shoup form
  const u64 *hat_mont; // [nin][nout]: (Qin/q_i mod r) 2^64 mod r
};

// ---------------------------------------------------------------- context

// A switching key's allocation: [dnum][2][L+1+K][N] Montgomery-form words,
// then the b halves again as 40-bit words (primes below 2^40), in a plane of
// low 32 bits [dnum][L+1+K][N] and a plane of high 8 bits of the same shape,
// so the kernels stream 5 bytes per b word instead of 8 on those limbs.
__host__ __device__ inline size_t key_words(int dnum, int keyl, int N) { return (size_t)dnum * 2 * keyl * N; }
__host__ __device__ inline size_t key_bytes(int dnum, int keyl, int N) {
  return key_words(dnum, keyl, N) * 8 + (((size_t)dnum * keyl * N * 5 + 7) & ~(size_t)7);
}
__device__ __forceinline__ u64 key_b40(const u64 *key, int dnum, int keyl, int N, int j, int p, int x) {
  const uint32_t *lo = (const uint32_t *)(key + key_words(dnum, keyl, N));
  const uint8_t *hi = (const uint8_t *)(lo + (size_t)dnum * keyl * N);
  const size_t i = ((size_t)j * keyl + p) * N + x;
  return (u64)lo[i] | ((u64)hi[i] << 32);
}

// Plaintext diagonals of a plan: [n_diag][L_pq][N] words in Montgomery form,
// then the same words as 40-bit values (a u32 low plane, then a u8 high
// plane), which the per-thread baby-step kernel reads on the limbs of primes
// below 2^40: 5 bytes a word instead of 8.
__host__ __device__ inline size_t pt_bytes(size_t words) { return words * 8 + ((words * 5 + 7) & ~(size_t)7); }
__device__ __forceinline__ u64 pt_b40(const u64 *pt, size_t words, size_t i) {
  const uint32_t *lo = (const uint32_t *)(pt + words);
  const uint8_t *hi = (const uint8_t *)(lo + words);
  return (u64)lo[i] | ((u64)hi[i] << 32);
}

struct KeyEntry {
  u64 *d;            // [dnum][2][L+1+K][N], Montgomery form
  u64 seed = 0;      // seed the a_j halves were expanded from
  bool seeded = false;
};

struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
  bool captured = false;   // a stream capture has used this allocation
};

// Kernel classes that can be timed with HIP events (helrm_timing_*).
enum TimedKernel {
  TK_NTT_FWD_COL = 0,
  TK_NTT_FWD_BLK,
  TK_NTT_INV_BLK,
  TK_NTT_INV_COL,
  TK_CONV,
  TK_KS_ACC,
  TK_BABY_MAC,
  TK_SUB_MUL,
  TK_BABY_MFMA,
  TK_BABY_FOLD,
  TK_COUNT
};

struct TimingRec {
  int k;
  hipEvent_t a, b;
  double bytes, ops;   // algorithmic bytes moved and modular products of this launch
};

struct helrm_ctx {
  int logn, N, L, K, alpha, dnum, nprimes;
  int device;
  std::vector<u64> primes;   // q_0..q_L, p_0..p_{K-1}
  std::vector<u64> psi;
  std::vector<PrimeInfo> h_pinfo;
  PrimeInfo *d_pinfo = nullptr;
  TW *d_tw_fwd = nullptr;    // [nprimes][N]: psi^brv(k)
  TW *d_tw_inv = nullptr;    // [nprimes][N]: psi^-brv(k)
  double *d_twd_fwd = nullptr;  // the same twiddles as doubles (exact for q < 2^45)
  double *d_twd_inv = nullptr;
  u64 *d_const = nullptr;    // conversion constants
  std::vector<std::vector<ConvTable>> modup_tabs;   // [level][digit]
  std::vector<ConvTable> moddown_tabs;              // [level]
  std::vector<const TW *> moddown_pinv;             // [level] -> [2][level+1] P^-1 mod q_i
  std::vector<const TW *> rescale_qinv;             // [level] -> [2][level] q_level^-1 mod q_i
  std::map<uint32_t, KeyEntry> keys;
  std::mutex ws_mu;
  std::map<hipStream_t, Workspace> ws;
  std::vector<void *> ws_retired;   // outgrown workspaces a captured graph may still use (freed at destroy)
  char *noalloc_scratch = nullptr;  // device address of this device's static scratch (helrm_lookup_packed_noalloc)
  int tune_ks_tile = 4;      // ciphertexts per thread in ks_acc (1, 2, 4)
  int tune_baby_tile = 4;    // ciphertexts per thread in baby_mac when one giant output (1, 2, 4)
  int tune_baby_share = 8;   // ciphertexts per workgroup in baby_mac with several giant outputs (1 = off, 2, 4, 8)
  int tune_ntt_col_w = 16;   // NTT column-pass columns per workgroup (8, 16; 0 = by launch size)
  int tune_ntt_blk_w = 4;    // NTT block-pass blocks per workgroup (4, 8; 0 = by launch size)
  int ntt_small_limbs = 48;  // launches of fewer limbs take the narrow shapes when a width is 0
  int tune_mfma_min_slots = 33;   // matrix-core MAC only for plans with at least this many baby steps
  int tune_fold_mp = 2;      // key-folded product: 2 row tiles per operand load (bit 0: 40-bit, bit 1: wide primes)
  int tune_block_chain = 1;   // key-folded product: workgroups in chain order of the coefficient blocks
  const u64 *d_block_chain = nullptr;   // [N/8]: block of 8 coefficients at chain position i (in d_const)
  const u64 *d_chain64 = nullptr;       // [N/64]: the same for blocks of 64 coefficients
  const u64 *d_chain256 = nullptr;      // [N/256]: and of 256
  int tune_ks_chain = 1;     // key-switching kernels: workgroups in chain order of their coefficient blocks
  int tune_limb_xcd = 0;      // key-switching kernels: whole limbs per XCD (1) or blocks dealt over the XCDs (0)
  int tune_fuse_ks = 1;       // ModDown fused with the ModUp or rescale that follows it (0 = off)
  int tune_fuse_conv = 1;   // fused boundary: c1's ModDown inside the ModUp conversions
  int tune_conv_wgs = 1536;  // base conversion: split outputs into chunks until a launch has this many workgroups (0 = off)
  int tune_baby_mfma = 8;    // batches of at least this many ciphertexts take the matrix-core plaintext MAC
                             // when the plan has its operands (0 = never)
  int tune_ptm = 1;          // plans with several giant steps build matrix-core operands (0 = never)
  int tune_baby_fold = 8;   // batches of at least this many ciphertexts take the key-folded matrix-core
                             // product when the plan has folded operands (0 = never)
  uint64_t keys_gen = 1;     // bumped by every helrm_load_eval_keys (folded operands of older keys are stale)
  int tune_gen_key_a = 1;    // regenerate keys' a_j halves from their seeds where a kernel serves one
                             // ciphertext per thread and streams keys: 0 never, 1 on primes below
                             // 2^40, 2 on every prime (default)
  bool timing = false;
  std::mutex tmu;
  std::vector<TimingRec> trecs;
  std::vector<hipEvent_t> evpool;

  int n_digits(int level) const { return (level + 1 + alpha - 1) / alpha; }
  int digit_lo(int j) const { return j * alpha; }
  int digit_hi(int j, int level) const {  // exclusive
    int h = (j + 1) * alpha;
    return h < level + 1 ? h : level + 1;
  }
  // index of the prime of PQ-limb r at this level
  int pq_prime(int r, int level) const { return r <= level ? r : L + 1 + (r - level - 1); }
  // position of PQ-limb r inside a full-level key
  int key_limb(int r, int level) const { return r <= level ? r : L + 1 + (r - level - 1); }
};

struct helrm_plan {
  helrm_ctx *ctx;
  int level, m, n1, n2, radix, n_diag, sign, span;
  std::vector<int> diag;                 // k = n1 g + b per stored diagonal
  std::vector<std::pair<int, int>> stages;  // fold (s, r)
  std::vector<int> babies;               // b values present (ascending)
  std::vector<int> giants;               // g values present (ascending)
  std::vector<int> slot;                 // [n2][n1]: stored diagonal index or -1
  u64 *d_pt = nullptr;                   // [n_diag][L_pq][N], Montgomery form, then its 40-bit planes
  size_t pt_words = 0;                   // n_diag * L_pq * N
  int *d_slot = nullptr;                 // device copy of slot
  size_t pt_limb_stride;                 // limbs per stored diagonal (= level+1+K)
  uint8_t *d_ptm = nullptr;              // matrix-core operands: [giant tile][L_pq][N] x 4 KiB (or null)
  int ptm_tiles = 0;
  // key-folded operands (helrm_plan_fold_keys): per giant tile, limb r and
  // coefficient x, wm_kc depth chunks of wm_planes[r] x 1 KiB; limb r starts
  // at wm_off[r] KiB-units x N x wm_kc within the tile
  uint8_t *d_wm = nullptr;
  int wm_kc = 0, wm_tiles = 0;
  size_t wm_tile_bytes = 0;
  std::vector<int> wm_planes, wm_off;
  uint64_t wm_keys_gen = 0;              // the context's key generation the operands were built from
};

// ---------------------------------------------------------------- timing

hipEvent_t timing_event(helrm_ctx *ctx);
void timing_push(helrm_ctx *ctx, int k, hipEvent_t a, hipEvent_t b, double bytes, double ops);

// Records a HIP event pair around one launch when timing is enabled.
struct KTimer {
  helrm_ctx *c;
  hipStream_t s;
  hipEvent_t a = nullptr;
  KTimer(helrm_ctx *ctx, hipStream_t st) : c(ctx), s(st) {
    if (c->timing) {
      a = timing_event(c);
      (void)hipEventRecord(a, s);
    }
  }
  // close the current interval as kernel class k and open the next one
  void lap(int k, double bytes, double ops) {
    if (!a) return;
    hipEvent_t b = timing_event(c);
    (void)hipEventRecord(b, s);
    timing_push(c, k, a, b, bytes, ops);
    a = b;
  }
};

// ---------------------------------------------------------------- launchers

#define HELRM_MAX_EPI 64

// Fused finish of a forward NTT: for list entries i < n_fin, instead of
// storing y = NTT(x), store out = (a - y) * c[i].  The transform's batch index
// splits into (outer, inner) = (bat / inner, bat % inner); a and out limbs
// live at outer * bs + inner * cs + off[i].  Entries i >= n_fin store y as
// usual and, where dup_off[i] >= 0, also at limb dup_off[i] of dup (batch
// stride dup_bs limbs).
struct NttEpi {
  const u64 *a = nullptr;
  u64 *out = nullptr;
  const TW *c = nullptr;
  int inner = 1;
  int n_fin = 0;
  int a_bs = 0, a_cs = 0, out_bs = 0, out_cs = 0;
  int a_off[HELRM_MAX_EPI] = {};
  int out_off[HELRM_MAX_EPI] = {};
  u64 *dup = nullptr;
  int dup_bs = 0;
  int dup_off[HELRM_MAX_LIMBS];
};

// NTT of the limbs in `ll` (src -> dst, may be in place).
int launch_ntt(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
               hipStream_t s);
int launch_ntt_epi(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                   hipStream_t s, const NttEpi &epi);

int launch_automorph(helrm_ctx *ctx, const u64 *in, u64 *out, uint32_t galois, int n_limbs, int batch,
                     hipStream_t s);
int launch_poly_op(helrm_ctx *ctx, int op, const u64 *a, const u64 *b, u64 *out, const LimbList &ll,
                   int batch, hipStream_t s);
int launch_mul_scalar(helrm_ctx *ctx, const u64 *a, const u64 *scal, u64 *out, const LimbList &ll,
                      int batch, hipStream_t s);
int launch_from_signed(helrm_ctx *ctx, const int64_t *in, u64 *out, const LimbList &ll, int batch,
                       hipStream_t s);
int launch_to_mont(helrm_ctx *ctx, u64 *data, const LimbList &ll, int batch, hipStream_t s);
// Fill a key's 40-bit planes of the b halves from its Montgomery-form words.
int launch_pack_pt(u64 *pt, size_t words, hipStream_t s);
int launch_pack_key(helrm_ctx *ctx, u64 *key, hipStream_t s);
int launch_copy_limbs(const u64 *src, u64 *dst, const LimbList &ll, int batch, int N, hipStream_t s);

// One fast base conversion (coefficient form) of a launch: inputs are the
// consecutive limbs src_off0.. of src, outputs go to dst_off[r]; ncopy limbs
// are copied unchanged from copy_src (evaluation-form own limbs of a digit).
// Finish of a P -> Q_l conversion done in coefficient form (ConvSpec::fin).
enum { CONV_FIN_NONE = 0, CONV_FIN_MODDOWN = 1, CONV_FIN_RESCALE = 2 };

struct ConvSpec {
  const ConvTable *t;
  int src_off0;
  int dst_off[HELRM_MAX_PRIMES];
  int ncopy = 0;
  int copy_src_off[16];
  int copy_dst_off[16];
  // CONV_FIN_MODDOWN: out_r = (A_r - conv_r) P^-1 mod q_r with A_r limb
  // fin_off0 + r of the source.  CONV_FIN_RESCALE: the same for every output,
  // then the rescale by the last output prime q_l; writes l outputs (qlinv:
  // q_l^-1 mod q_r, r < l).
  int fin = CONV_FIN_NONE;
  int fin_off0 = 0;
  const TW *qlinv = nullptr;
  // A ModDown in front (fused boundary, pre = table of the ModDown P -> Q_l,
  // whose number of special primes equals this job's input count): input i
  // is not read but formed as z_i = (A_i - conv_{c_i}) P^-1 mod q_i, conv
  // the conversion of the special limbs pre_src0 + k of the source to Q limb
  // c_i = pre_col0 + i, A_i the coefficient-form Q limb pre_a0 + i of the
  // source; z_i is also written to limb pre_dst0 + i of the destination.
  const ConvTable *pre = nullptr;
  int pre_src0 = 0, pre_a0 = 0, pre_col0 = 0, pre_dst0 = 0;
};
int launch_conv(helrm_ctx *ctx, const ConvSpec *specs, int nspecs, const u64 *src, int src_bstride,
                const u64 *copy_src, int copy_bstride, u64 *dst, int dst_bstride, int batch, hipStream_t s);

// out[l] = (a[l] - b[l]) * consts[l]  (consts: Shoup pairs, one per list entry)
// b is addressed with the dst offsets of ll and batch stride b_bstride.
int launch_sub_mul(helrm_ctx *ctx, const u64 *a, const u64 *b, int b_bstride, u64 *out,
                   const LimbList &ll, const TW *consts, int batch, hipStream_t s);

// Rescale middle step: from the coefficient-form top limb c (both polys),
// write [ (c + h mod q_l) - h ]_{q_i} for i < level.
int launch_rescale_spread(helrm_ctx *ctx, const u64 *top, u64 *out, int level, int batch,
                          hipStream_t s);

struct KsTerm {
  const u64 *digits;  // [beta][level+1+K][N] (batch stride given separately)
  const u64 *c0;      // [level+1][N], or null: no P sigma(c0) term
  const u64 *key;     // [dnum][2][L+1+K][N] Montgomery form
  uint32_t galois;
  u64 seed = 0;       // the key's seed, when its a_j halves may be regenerated
  bool seeded = false;
};

// 5^(step mod n) mod 2N by square-and-multiply (2N is a power of two).
inline uint32_t galois_of_step(const helrm_ctx *ctx, long step) {
  const long n = ctx->N / 2;
  unsigned long k = (unsigned long)(((step % n) + n) % n);
  const u64 mask = 2ull * ctx->N - 1;
  u64 g = 1, b = 5;
  for (; k; k >>= 1, b = b * b & mask)
    if (k & 1) g = g * b & mask;
  return (uint32_t)g;
}

// Plain a_j of a seeded key over every prime of PQ_L: out [L+1+K][N].
int launch_key_uniform(helrm_ctx *ctx, u64 seed, int digit, u64 *out, hipStream_t s);

// Matrix-core operands of a plan (giant tiles of 8, at most 64 baby steps
// per tile): slot_tab [tiles][64][8] device array of stored diagonal indices.
int launch_ptm_pack(helrm_ctx *ctx, const helrm_plan *plan, const int *slot_tab, hipStream_t s);

// 32-bit words of the folded product's entry workspace per ciphertext at a
// level (entries of the rotated steps, then of step 0): 2 N sum_r P_r.
inline size_t fold_entry_words(const helrm_ctx *ctx, int level) {
  size_t tot = 0;
  for (int r = 0; r < level + 1 + ctx->K; r++) tot += ctx->primes[ctx->pq_prime(r, level)] < (1ull << 40) ? 5 : 8;
  return 2 * tot * (size_t)ctx->N;
}

// Key-folded operands of giant tile T of a plan (helrm_plan_fold_keys).
int launch_wfold_pack(helrm_ctx *ctx, helrm_plan *plan, int T, hipStream_t s);

// ALU calibration (measurement only; both block until done): butterflies per
// second of the NTT arithmetic on prime q, and instructions per second of
// v_mad_u64_u32 (kind 0) or fp64 FMA (kind 1), counted per lane.
int calibrate_butterflies(helrm_ctx *ctx, u64 q, hipStream_t s, double *per_s);
int calibrate_instr(int kind, hipStream_t s, double *per_s);
// (d0, d1, d2) of two ciphertexts at `level` ([batch][2][level+1] -> [batch][3][level+1]).
int launch_tensor(helrm_ctx *ctx, const u64 *a, const u64 *b, u64 *d, int level, int batch, hipStream_t s);
// (c0 + pt, c1) with one plaintext [level+1] limbs for every ciphertext of the batch.
int launch_add_plain(helrm_ctx *ctx, const u64 *ct, const u64 *pt, u64 *out, int level, int batch,
                     hipStream_t s);

// out (PQ, 2 polys) = [lift_P(base)] + sum_t KeyIP(term t).
int launch_ks_accumulate(helrm_ctx *ctx, int level, const KsTerm *terms, int n_terms,
                         size_t digits_bstride, size_t c0_bstride, const u64 *base,
                         size_t base_bstride, u64 *out, size_t out_bstride, int batch, hipStream_t s);

// Fused baby steps + plaintext MAC: X_g = sum_b pt_{g,b} (.) R_b for g in
// [g0, g0+ng).
// accum: add to what X holds; force: launch (writing zeros) even when no baby
// step of this plan feeds giants g0..g0+ng-1; fold_ws: batch x
// fold_entry_words(level) words of workspace for the key-folded product
// (null: that product is not taken).
int launch_baby_mac(helrm_ctx *ctx, const helrm_plan *plan, const u64 *digits, size_t digits_bstride,
                    const u64 *ct, size_t ct_bstride, u64 *X, size_t x_bstride, int g0, int ng,
                    int batch, hipStream_t s, bool accum = false, bool force = false,
                    uint32_t *fold_ws = nullptr);
