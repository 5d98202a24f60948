// Element-wise, automorphism, base-conversion, rescale and key-switching
// kernels of libhelrm (gfx950).  All residues are uint64; one thread owns one
// coefficient position of one limb, so every global access is a coalesced
// run of consecutive words (the automorphism gathers inside aligned blocks:
// X -> X^g maps each aligned block of 2^k evaluation points onto an aligned
// block of 2^k points).
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ size_t limb_ptr(int bat, int bstride, int off, int N) {
  return ((size_t)bat * bstride + off) * (size_t)N;
}

// ---------------------------------------------------------------- element-wise

__global__ __launch_bounds__(TPB) void poly_op_kernel(int op, const u64 *a, const u64 *b, u64 *out,
                                                      LimbList ll, const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  const PrimeInfo pi = pinfo[ll.prime[li]];
  const size_t ia = limb_ptr(bat, ll.src_bstride, ll.src_off[li], N) + x;
  const size_t io = limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x;
  const u64 va = a[ia];
  u64 r;
  if (op == HELRM_OP_NEG) {
    r = va == 0 ? 0 : pi.q - va;
  } else {
    const u64 vb = b[ia];
    if (op == HELRM_OP_ADD) {
      r = add_mod(va, vb, pi.q);
    } else if (op == HELRM_OP_SUB) {
      r = sub_mod(va, vb, pi.q);
    } else {
      u128 p = (u128)va * vb;
      u64 t = redc((u64)p, (u64)(p >> 64), pi.q, pi.qn);   // a b 2^-64
      p = (u128)t * pi.r2;
      r = redc((u64)p, (u64)(p >> 64), pi.q, pi.qn);       // a b
    }
  }
  out[io] = r;
}

struct ScalarArgs {
  TW c[64];
};

__global__ __launch_bounds__(TPB) void mul_scalar_kernel(const u64 *a, u64 *out, LimbList ll,
                                                         ScalarArgs sc, const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  const u64 q = pinfo[ll.prime[li]].q;
  const size_t ia = limb_ptr(bat, ll.src_bstride, ll.src_off[li], N) + x;
  const size_t io = limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x;
  out[io] = shoup(a[ia], sc.c[li].w, sc.c[li].wp, q);
}

__global__ __launch_bounds__(TPB) void from_signed_kernel(const int64_t *in, u64 *out, LimbList ll,
                                                          const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  const PrimeInfo pi = pinfo[ll.prime[li]];
  const int64_t v = in[(size_t)bat * N + x];
  const u64 mag = v >= 0 ? (u64)v : (u64)(-(v + 1)) + 1u;
  u64 r = reduce64(mag, pi.q, pi.mu);
  if (v < 0 && r != 0) r = pi.q - r;
  out[limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x] = r;
}

__global__ __launch_bounds__(TPB) void to_mont_kernel(u64 *data, LimbList ll, const PrimeInfo *pinfo,
                                                      int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  const PrimeInfo pi = pinfo[ll.prime[li]];
  const size_t i = limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x;
  u128 p = (u128)data[i] * pi.r2;
  data[i] = redc((u64)p, (u64)(p >> 64), pi.q, pi.qn);
}

__global__ __launch_bounds__(TPB) void copy_limbs_kernel(const u64 *src, u64 *dst, LimbList ll, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  dst[limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x] =
      src[limb_ptr(bat, ll.src_bstride, ll.src_off[li], N) + x];
}

__global__ __launch_bounds__(TPB) void automorph_kernel(const u64 *in, u64 *out, unsigned g, int logn) {
  const int N = 1 << logn;
  const int x = blockIdx.x * TPB + threadIdx.x;
  const size_t base = (size_t)blockIdx.y * N;
  out[base + x] = in[base + galois_src(x, g, logn)];
}

// out[l] = (a[l] - b[l]) * c[l]  with c in Shoup form (ModDown: P^-1,
// rescale: q_l^-1).  a uses the src offsets, b and out the dst offsets.
__global__ __launch_bounds__(TPB) void sub_mul_kernel(const u64 *a, const u64 *b, u64 *out, LimbList ll,
                                                      const TW *consts, const PrimeInfo *pinfo, int N,
                                                      int b_bstride) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % ll.n, bat = blockIdx.y / ll.n;
  const u64 q = pinfo[ll.prime[li]].q;
  const u64 va = a[limb_ptr(bat, ll.src_bstride, ll.src_off[li], N) + x];
  const u64 vb = b[limb_ptr(bat, b_bstride, ll.dst_off[li], N) + x];
  const TW c = consts[li];
  out[limb_ptr(bat, ll.dst_bstride, ll.dst_off[li], N) + x] = shoup(sub_mod(va, vb, q), c.w, c.wp, q);
}

// ---------------------------------------------------------------- base conversion

// One base conversion job of a launch: the input limbs are consecutive
// (src_off0 + i), the outputs go to arbitrary limb offsets; optionally the
// job also copies `ncopy` limbs unchanged (ModUp: each digit's own limbs,
// already in evaluation form, from copy_src).
struct ConvJob {
  ConvTable t;
  int src_off0;
  int dst_off[HELRM_MAX_PRIMES];
  int ncopy;
  int copy_src_off[16];
  int copy_dst_off[16];
  int fin;            // CONV_FIN_* (ConvSpec)
  int fin_off0;       // A_r is limb fin_off0 + r of src
  const TW *qlinv;    // CONV_FIN_RESCALE: q_l^-1 mod q_r for r < l
  // ModDown in front (ConvSpec::pre): special primes pre_prime0 + k, their
  // (P/p_k)^-1 mod p_k and the [K][pre_ncol] Montgomery-form [P/p_k]_q matrix
  int pre;            // 0: inputs read from src
  int pre_src0, pre_a0, pre_col0, pre_dst0, pre_ncol, pre_prime0;
  const TW *pre_hat_inv;
  const u64 *pre_hat_mont;
};

struct ConvJobs {
  int njobs;
  int nchunks;       // output chunks per job (the last one also copies)
  ConvJob j[HELRM_MAX_CONV_JOBS];
};

constexpr int CONV_TPB = 256;

// y_i = x_i (Qin/q_i)^-1 mod q_i;  out_r = sum_i y_i [Qin/q_i]_r mod r, the
// sum of NIN <= 16 products formed in 30-bit halves (Sum30) and finished by
// one REDC (the constants are in Montgomery form).  A thread owns one coefficient and one chunk of the outputs (J.nchunks
// chunks per job; the copies are dealt round-robin over the chunks).  Small
// launches (batch 1: a few hundred coefficient blocks) split the outputs so
// every SIMD holds several waves; each chunk re-reads the NIN inputs, which
// the neighbouring workgroups of the same coefficient block (consecutive
// block indices) find in L2.  The [NIN][nout] constant matrix is staged in
// LDS and read as broadcasts.  Grid: (N/CONV_TPB * nchunks, 1, batch * njobs).
//
// With a finish (ModDown in coefficient form, the conversion being P -> Q_l)
// output r becomes z_r = (A_r - out_r) P^-1 mod q_r, A_r the coefficient-form
// Q limb of the input; with the rescale as well, every chunk also forms the
// top output z_l and writes (z_r - [t - h]_{q_r}) q_l^-1 for r < l, where
// t = (z_l + h) mod q_l and h = floor(q_l / 2) (rounding division by q_l).
// With a ModDown in front (a ModUp digit of a fused boundary; PRE kernels)
// the thread forms the digit's inputs z_i from the special limbs in the same
// way and writes them; the ModDown's own launch and the re-read of z are
// saved.  Such launches are not split into output chunks (each chunk would
// form z again).
template <int NIN, bool PRE>
__global__ __launch_bounds__(CONV_TPB) void conv_kernel(const ConvJobs J, const u64 *src, int src_bstride,
                                                        const u64 *copy_src, int copy_bstride, u64 *dst,
                                                        int dst_bstride, const PrimeInfo *pinfo, int N) {
  __shared__ u64 cm[NIN * HELRM_MAX_PRIMES];
  __shared__ u64 cpre[PRE ? NIN * NIN : 1];
  __shared__ u64 oq[HELRM_MAX_PRIMES], oqn[HELRM_MAX_PRIMES], opi[HELRM_MAX_PRIMES], opp[HELRM_MAX_PRIMES],
      omu[HELRM_MAX_PRIMES];
  const int chunk = blockIdx.x % J.nchunks;
  const int x = (blockIdx.x / J.nchunks) * CONV_TPB + threadIdx.x;
  const int job = blockIdx.z % J.njobs, bat = blockIdx.z / J.njobs;
  const ConvJob &jb = J.j[job];
  const int nout = jb.t.nout;
  const int fin = jb.fin;
  const int nw = fin == CONV_FIN_RESCALE ? nout - 1 : nout;   // outputs written
  const int per = (nw + J.nchunks - 1) / J.nchunks;
  const int r0 = chunk * per, r1 = min(nw, r0 + per);
  // inputs of this job: a PRE launch may mix jobs of NIN and fewer inputs
  // (the missing ones enter as zero), the others have NIN each
  const int nin = PRE ? jb.t.nin : NIN;
  for (int k = threadIdx.x; k < nin * nout; k += CONV_TPB) cm[k] = split30(jb.t.hat_mont[k]);
  if (PRE && jb.pre)
    for (int k = threadIdx.x; k < NIN * NIN; k += CONV_TPB)
      cpre[k] = k % NIN < nin ? split30(jb.pre_hat_mont[(k / NIN) * jb.pre_ncol + jb.pre_col0 + k % NIN]) : 0;
  for (int k = threadIdx.x; k < nout; k += CONV_TPB) {
    const PrimeInfo &po = pinfo[jb.t.out_prime[k]];
    oq[k] = po.q;
    oqn[k] = po.qn;
    opi[k] = po.pinv;
    opp[k] = po.pinv_p;
    omu[k] = po.mu;
  }
  u64 y[NIN];
  if (PRE && jb.pre) {
    // the special limbs, (P/p_k)^-1 applied
    u64 yp[NIN];
#pragma unroll
    for (int k = 0; k < NIN; k++) {
      const u64 q = pinfo[jb.pre_prime0 + k].q;
      const u64 v = src[limb_ptr(bat, src_bstride, jb.pre_src0 + k, N) + x];
      yp[k] = split30(shoup(v, jb.pre_hat_inv[k].w, jb.pre_hat_inv[k].wp, q));
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NIN; i++) {
      y[i] = 0;
      if (i < nin) {
        const PrimeInfo &pq = pinfo[jb.t.in_prime[i]];
        Sum30 a;
        a.zero();
#pragma unroll
        for (int k = 0; k < NIN; k++) a.mac(yp[k], cpre[k * NIN + i]);
        const u64 A = src[limb_ptr(bat, src_bstride, jb.pre_a0 + i, N) + x];
        const u64 z = shoup(sub_mod(A, redc_acc(a.value(), pq.q, pq.qn), pq.q), pq.pinv, pq.pinv_p, pq.q);
        if (chunk == 0) dst[limb_ptr(bat, dst_bstride, jb.pre_dst0 + i, N) + x] = z;
        y[i] = split30(shoup(z, jb.t.hat_inv[i].w, jb.t.hat_inv[i].wp, pq.q));
      }
    }
  } else {
    if (r0 < r1) {
#pragma unroll
      for (int i = 0; i < NIN; i++) {
        y[i] = 0;
        if (i < nin) {
          const u64 q = pinfo[jb.t.in_prime[i]].q;
          const u64 v = src[limb_ptr(bat, src_bstride, jb.src_off0 + i, N) + x];
          y[i] = split30(shoup(v, jb.t.hat_inv[i].w, jb.t.hat_inv[i].wp, q));
        }
      }
    }
    __syncthreads();
  }
  // converted (and finished) output r
  auto outv = [&](int r) -> u64 {
    Sum30 a;
    a.zero();
#pragma unroll
    for (int i = 0; i < NIN; i++) a.mac(y[i], cm[i * nout + r]);
    u64 v = redc_acc(a.value(), oq[r], oqn[r]);
    if (fin != CONV_FIN_NONE) {
      const u64 A = src[limb_ptr(bat, src_bstride, jb.fin_off0 + r, N) + x];
      v = shoup(sub_mod(A, v, oq[r]), opi[r], opp[r], oq[r]);
    }
    return v;
  };
  if (fin == CONV_FIN_RESCALE) {
    if (r0 < r1) {
      const int top = nout - 1;
      const u64 ql = oq[top], h = ql >> 1;
      u64 t = outv(top) + h;
      t = t >= ql ? t - ql : t;
      for (int r = r0; r < r1; r++) {
        const u64 q = oq[r];
        u64 sp;
        if (t >= h) {
          sp = reduce64(t - h, q, omu[r]);
        } else {
          sp = reduce64(h - t, q, omu[r]);
          sp = sp == 0 ? 0 : q - sp;
        }
        const TW c = jb.qlinv[r];
        dst[limb_ptr(bat, dst_bstride, jb.dst_off[r], N) + x] = shoup(sub_mod(outv(r), sp, q), c.w, c.wp, q);
      }
    }
  } else {
    for (int r = r0; r < r1; r++) dst[limb_ptr(bat, dst_bstride, jb.dst_off[r], N) + x] = outv(r);
  }
  for (int c = chunk; c < jb.ncopy; c += J.nchunks)
    dst[limb_ptr(bat, dst_bstride, jb.copy_dst_off[c], N) + x] =
        copy_src[limb_ptr(bat, copy_bstride, jb.copy_src_off[c], N) + x];
}

// Rescale middle step: t = (c + h) mod q_l from the top limb (coefficient
// form), then [t - h]_{q_i} for every lower prime i.
__global__ __launch_bounds__(TPB) void rescale_spread_kernel(const u64 *top, u64 *out, int level,
                                                             const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int i = blockIdx.y % level, cb = blockIdx.y / level;   // cb = bat*2 + poly
  const u64 ql = pinfo[level].q;
  const u64 h = ql >> 1;
  u64 t = top[(size_t)cb * N + x] + h;
  t = t >= ql ? t - ql : t;
  const PrimeInfo pi = pinfo[i];
  u64 r;
  if (t >= h) {
    r = reduce64(t - h, pi.q, pi.mu);
  } else {
    r = reduce64(h - t, pi.q, pi.mu);
    r = r == 0 ? 0 : pi.q - r;
  }
  out[((size_t)cb * level + i) * N + x] = r;
}

// ---------------------------------------------------------------- ciphertext products and additions

// (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) per limb, canonical residues.
// a, b: [batch][2][qn] limbs; d: [batch][3][qn].  Each product is a REDC of a
// 128-bit sum (a b 2^-64) followed by a REDC with 2^128 mod q.
__global__ __launch_bounds__(TPB) void tensor_kernel(const u64 *a, const u64 *b, u64 *d, int qn,
                                                     const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int r = blockIdx.y % qn, bat = blockIdx.y / qn;
  const PrimeInfo pi = pinfo[r];
  const size_t ia = ((size_t)bat * 2 * qn + r) * N + x, off1 = (size_t)qn * N;
  const u64 a0 = a[ia], a1 = a[ia + off1], b0 = b[ia], b1 = b[ia + off1];
  auto finish = [&](const Acc &s) {
    const u64 t = redc_acc(s, pi.q, pi.qn);
    const u128 p = (u128)t * pi.r2;
    return redc((u64)p, (u64)(p >> 64), pi.q, pi.qn);
  };
  Acc s0, s1, s2;
  acc_zero(s0);
  acc_zero(s1);
  acc_zero(s2);
  acc_mac(s0, a0, b0);
  acc_mac(s1, a0, b1);
  acc_mac(s1, a1, b0);
  acc_mac(s2, a1, b1);
  const size_t id = ((size_t)bat * 3 * qn + r) * N + x;
  d[id] = finish(s0);
  d[id + off1] = finish(s1);
  d[id + 2 * off1] = finish(s2);
}

// out = (c0 + pt, c1); ct, out: [batch][2][qn] limbs; pt: [qn] limbs, shared.
__global__ __launch_bounds__(TPB) void add_plain_kernel(const u64 *ct, const u64 *pt, u64 *out, int qn,
                                                        const PrimeInfo *pinfo, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int li = blockIdx.y % (2 * qn), bat = blockIdx.y / (2 * qn);
  const size_t i = ((size_t)bat * 2 * qn + li) * N + x;
  if (li < qn)
    out[i] = add_mod(ct[i], pt[(size_t)li * N + x], pinfo[li].q);
  else
    out[i] = ct[i];
}

// ---------------------------------------------------------------- key switching

struct KsArgs {
  int n;
  int accum;   // add the result to what `out` holds (later chunks of a long term list)
  u64 seed[HELRM_MAX_TERMS];   // key seeds (used when the a_j halves are regenerated)
  const u64 *digits[HELRM_MAX_TERMS];
  const u64 *c0[HELRM_MAX_TERMS];
  const u64 *key[HELRM_MAX_TERMS];
  unsigned gal[HELRM_MAX_TERMS];
};

struct LevelGeom {
  int level, beta, pqn, keyl, logn;
  int keyd;       // digits of a stored key (dnum), for the 40-bit planes of its b halves
  int limb_xcd;   // tile_map: whole limbs per XCD (1) or blocks dealt over the XCDs (0)
  int gen_wide;   // kernels that regenerate key halves do so on primes >= 2^40 too (1)
  const u64 *chain = nullptr;   // workgroup order (chain_map) of the launch's coefficient blocks, or none
};

__device__ __forceinline__ int pq_prime_dev(int r, int level, int L) {
  return r <= level ? r : L + 1 + (r - level - 1);
}

// Workgroup order of the key-switching kernels.  A group is one block of
// coefficients of one limb (nx blocks per limb, nr limbs), a tile is one
// slice of the batch; workgroup L runs on XCD L mod 8 (round-robin dispatch)
// and each XCD starts its workgroups in order.  With limb_xcd, limb r of the
// first 8 floor(nr/8) limbs is served by XCD r mod 8 alone, group by group,
// the tiles of a group back to back: the rotations of a limb gather its
// digit and c0 words from the blocks the Galois map sends them to (a
// 64-aligned block of slots maps onto another one), so after the first
// rotation they come from that XCD's L2, and the key and plaintext words of a
// group serve every tile from L2 as well.  The other nr mod 8 limbs (and
// every limb without limb_xcd) are dealt over the XCDs group by group.
struct TileMap {
  int xb, r, tile;
};

__device__ __forceinline__ TileMap tile_map(int L, int nx, int ntiles, int nr, int limb_xcd) {
  const int xcd = L & 7, k = L >> 3;
  const int nr8 = limb_xcd ? (nr & ~7) : 0;
  const int first = (nr8 >> 3) * nx * ntiles;   // workgroups per XCD on whole limbs
  TileMap m;
  if (k < first) {
    const int g = k / ntiles;
    m.tile = k % ntiles;
    m.xb = g % nx;
    m.r = (g / nx) * 8 + xcd;
  } else {
    const int k2 = k - first;
    const int grp = (k2 / ntiles) * 8 + xcd;
    m.tile = k2 % ntiles;
    m.xb = grp % nx;
    m.r = nr8 + grp / nx;
  }
  return m;
}

// Workgroup order along a chain of coefficient blocks.  A block of 2^k
// consecutive coefficients (evaluation points with exponents e = 2 brv(x) +
// 1) is one class of e modulo 2N / 2^k, and every Galois map sends a block
// onto a block; the rotation by 5^b sends the block of class ±5^i to that of
// ±5^(i+b).  The chain lists the blocks in the order of i (the two signs one
// after the other), so a rotation shifts chain positions by b.  XCD x takes
// the x-th eighth of the chain positions of every limb, limb by limb (and
// the ciphertext tiles of a position back to back): the workgroups resident
// on one XCD then gather their rotated words from a window of a few times
// the rotation count of blocks, which stays in that XCD's L2, and every XCD
// gets the same mix of cheap and costly (wide-prime) limbs.  Without a
// chain: the key-switching kernels' order above.
__device__ __forceinline__ TileMap chain_map(int L, int nx, int ntiles, int nr, int limb_xcd, const u64 *chain) {
  if (!chain) return tile_map(L, nx, ntiles, nr, limb_xcd);
  const int xcd = L & 7, k = L >> 3;
  const int pe = nx >> 3;                 // chain positions per XCD and limb (nx is a multiple of 8)
  const int per_limb = pe * ntiles;
  const int w = k % per_limb;
  TileMap m;
  m.r = k / per_limb;
  m.tile = w % ntiles;
  m.xb = (int)chain[xcd * pe + w / ntiles];
  return m;
}

constexpr int MAXBETA = 4;   // digits per key switch handled in registers

// Multiply-accumulate policy of limbs with primes of 40 bits and more: the
// four-multiply Wide30Mac where a thread holds at most two accumulator pairs,
// the four-register WideMac otherwise.
template <int TILES>
using WideOf = typename std::conditional<(TILES <= 2), Wide30Mac, WideMac>::type;

// out = (B, A) over PQ:  B = sum_t sum_j sigma_t(d_{t,j}) b_{t,j}
//                          + P (sum_t sigma_t(c0_t) + base_c0),
//                        A = sum_t sum_j sigma_t(d_{t,j}) a_{t,j} + P base_c1.
// Each thread owns one coefficient of one limb for BT ciphertexts; the key
// words of a rotation are loaded once and used for all BT.  The loads of the
// next term are issued before the products of the current one.
template <int BT, int BETA>
struct KsIn {
  u64 kb[BETA], ka[BETA], d[BT][BETA], c0[BT];
};

template <int BT, int BETA, class M, bool GEN>
__device__ __forceinline__ void ks_acc_body(const KsArgs &T, const LevelGeom &G, int batch, int x, int r, int b0,
                                            int p, const PrimeInfo &pi, size_t dig_bs, size_t c0_bs,
                                            const u64 *base, size_t base_bs, u64 *out, size_t out_bs) {
  const int N = 1 << G.logn;
  constexpr bool NARROW = std::is_same<M, SplitMac>::value;   // prime below 2^40: b halves from the 40-bit planes
  const bool isq = r <= G.level;
  const int nct = min(BT, batch - b0);
  M ab[BT], aa[BT];
  u64 csum[BT];
#pragma unroll
  for (int k = 0; k < BT; k++) {
    ab[k].zero();
    aa[k].zero();
    csum[k] = 0;
  }
  auto load = [&](KsIn<BT, BETA> &in, int t) {
    const unsigned src = galois_src(x, T.gal[t], G.logn);
    const u64 *kk = T.key[t];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
      in.kb[j] = NARROW ? key_b40(kk, G.keyd, G.keyl, N, j, p, x) : kk[((size_t)(2 * j) * G.keyl + p) * N + x];
      in.ka[j] = GEN ? key_uniform_mont(T.seed[t], j, p, x, pi) : kk[((size_t)(2 * j + 1) * G.keyl + p) * N + x];
    }
#pragma unroll
    for (int k = 0; k < BT; k++) {
      if (k < nct) {
        const u64 *dg = T.digits[t] + (b0 + k) * dig_bs;
#pragma unroll
        for (int j = 0; j < BETA; j++) in.d[k][j] = dg[((size_t)j * G.pqn + r) * N + src];
        in.c0[k] = isq && T.c0[t] ? T.c0[t][(b0 + k) * c0_bs + (size_t)r * N + src] : 0;
      }
    }
  };
  auto step = [&](const KsIn<BT, BETA> &in) {
    typename M::Op kb[BETA], ka[BETA];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
      kb[j] = M::prep(in.kb[j]);
      ka[j] = M::prep(in.ka[j]);
    }
#pragma unroll
    for (int k = 0; k < BT; k++) {
      if (k < nct) {
#pragma unroll
        for (int j = 0; j < BETA; j++) {
          const auto d = M::prep(in.d[k][j]);
          ab[k].mac(d, kb[j]);
          aa[k].mac(d, ka[j]);
        }
        if (isq) csum[k] = add_mod(csum[k], in.c0[k], pi.q);
      }
    }
  };
  KsIn<BT, BETA> A, B;
  if (T.n > 0) load(A, 0);
  for (int t = 0; t < T.n; t += 2) {
    if (t + 1 < T.n) load(B, t + 1);
    step(A);
    if (t + 1 >= T.n) break;
    if (t + 2 < T.n) load(A, t + 2);
    step(B);
  }
#pragma unroll
  for (int k = 0; k < BT; k++) {
    if (k >= nct) break;
    const int bat = b0 + k;
    u64 Bv = ab[k].finish(pi.q, pi.qn);
    u64 Av = aa[k].finish(pi.q, pi.qn);
    u64 cs = csum[k];
    if (isq) {
      if (base) {
        const u64 *bb = base + bat * base_bs;
        cs = add_mod(cs, bb[(size_t)r * N + x], pi.q);
        Av = add_mod(Av, shoup(bb[((size_t)(G.level + 1) + r) * N + x], pi.pmod, pi.pmod_p, pi.q), pi.q);
      }
      Bv = add_mod(Bv, shoup(cs, pi.pmod, pi.pmod_p, pi.q), pi.q);
    }
    u64 *o = out + bat * out_bs;
    if (T.accum) {
      Bv = add_mod(Bv, o[(size_t)r * N + x], pi.q);
      Av = add_mod(Av, o[((size_t)G.pqn + r) * N + x], pi.q);
    }
    o[(size_t)r * N + x] = Bv;
    o[((size_t)G.pqn + r) * N + x] = Av;
  }
}

template <int BT, int BETA, bool GEN>
__global__ __launch_bounds__(TPB) void ks_acc_kernel(KsArgs T, LevelGeom G, int L, int batch, int ntiles,
                                                     size_t dig_bs, size_t c0_bs, const u64 *base,
                                                     size_t base_bs, u64 *out, size_t out_bs,
                                                     const PrimeInfo *pinfo) {
  const int N = 1 << G.logn;
  const TileMap tm = chain_map(blockIdx.x, N / TPB, ntiles, G.pqn, G.limb_xcd, G.chain);
  const int x = tm.xb * TPB + threadIdx.x;
  const int p = pq_prime_dev(tm.r, G.level, L);
  const PrimeInfo pi = pinfo[p];
  if (pi.q < SPLIT_MAC_LIMIT)
    ks_acc_body<BT, BETA, SplitMac, GEN>(T, G, batch, x, tm.r, tm.tile * BT, p, pi, dig_bs, c0_bs, base, base_bs,
                                         out, out_bs);
  else if (GEN && G.gen_wide)
    ks_acc_body<BT, BETA, WideOf<BT>, GEN>(T, G, batch, x, tm.r, tm.tile * BT, p, pi, dig_bs, c0_bs, base,
                                           base_bs, out, out_bs);
  else
    ks_acc_body<BT, BETA, WideOf<BT>, false>(T, G, batch, x, tm.r, tm.tile * BT, p, pi, dig_bs, c0_bs, base,
                                             base_bs, out, out_bs);
}

// Rotation steps of one fused baby-step launch, compacted on the host: only
// baby steps that some giant output of the launch uses are listed.
struct BabyArgs {
  int nrot;                                        // rotation steps (b > 0)
  int has0;                                        // b = 0 contributes
  short slot0[HELRM_MAX_GTILE];                    // plaintext of (g0 + gi, b = 0), -1: none
  unsigned gal[HELRM_MAX_BABY];                    // Galois element of each step
  const u64 *key[HELRM_MAX_BABY];                  // its evaluation key
  u64 seed[HELRM_MAX_BABY];                        // the key's seed (a_j regenerated from it)
  short slot[HELRM_MAX_BABY][HELRM_MAX_GTILE];     // plaintext of (g0 + gi, step), -1: none
};

// Loads of one rotation step for BT ciphertexts and GT giant outputs.
template <int GT, int BT, int BETA>
struct StepIn {
  u64 kb[BETA], ka[BETA], d[BT][BETA], c0[BT], w[GT];
};

// Fused hoisted baby-step rotations and plaintext-diagonal MAC (double
// hoisting): R_b is formed in registers and immediately multiplied into every
// giant output of the tile, so no rotated ciphertext is written to memory.
// Each thread serves BT ciphertexts: key and plaintext words are loaded once
// per rotation and reused for all of them.  The loads of the next rotation
// step are issued before the products of the current one.  M is the
// multiply-accumulate policy (SplitMac on limbs whose prime is below 2^40,
// WideMac otherwise); BETA is the number of key-switching digits.
template <int GT, int BT, int BETA, class M, bool GEN>
__device__ __forceinline__ void baby_mac_body(const BabyArgs &BA, const LevelGeom &G, int batch, int x, int r,
                                              int b0, int p, const PrimeInfo &pi, const u64 *digits,
                                              size_t dig_bs, const u64 *ct, size_t ct_bs, const u64 *pt,
                                              size_t pt_words, int ng, u64 *X, size_t x_bs, int accum) {
  const int N = 1 << G.logn;
  // prime below 2^40: key b halves and plaintexts from their 40-bit planes
  constexpr bool NARROW = std::is_same<M, SplitMac>::value;
  auto ptw = [&](int s) -> u64 {
    const size_t i = ((size_t)s * G.pqn + r) * N + x;
    return NARROW ? pt_b40(pt, pt_words, i) : pt[i];
  };
  const bool isq = r <= G.level;
  const int nct = min(BT, batch - b0);
  M acc[BT][GT][2];
#pragma unroll
  for (int k = 0; k < BT; k++)
#pragma unroll
    for (int gi = 0; gi < GT; gi++) {
      acc[k][gi][0].zero();
      acc[k][gi][1].zero();
    }
  if (BA.has0 && isq) {
    typename M::Op w[GT];
#pragma unroll
    for (int gi = 0; gi < GT; gi++) {
      const int s = gi < ng ? BA.slot0[gi] : -1;
      w[gi] = M::prep(s >= 0 ? ptw(s) : 0);
    }
#pragma unroll
    for (int k = 0; k < BT; k++) {
      if (k < nct) {
        const u64 *c = ct + (b0 + k) * ct_bs;
        const auto RB = M::prep(shoup(c[(size_t)r * N + x], pi.pmod, pi.pmod_p, pi.q));
        const auto RA = M::prep(shoup(c[((size_t)(G.level + 1) + r) * N + x], pi.pmod, pi.pmod_p, pi.q));
#pragma unroll
        for (int gi = 0; gi < GT; gi++) {
          acc[k][gi][0].mac(w[gi], RB);
          acc[k][gi][1].mac(w[gi], RA);
        }
      }
    }
  }
  auto load = [&](StepIn<GT, BT, BETA> &in, int i) {
    const unsigned src = galois_src(x, BA.gal[i], G.logn);
    const u64 *kk = BA.key[i];
#pragma unroll
    for (int j = 0; j < BETA; j++) {
      in.kb[j] = NARROW ? key_b40(kk, G.keyd, G.keyl, N, j, p, x) : kk[((size_t)(2 * j) * G.keyl + p) * N + x];
      in.ka[j] = GEN ? key_uniform_mont(BA.seed[i], j, p, x, pi) : kk[((size_t)(2 * j + 1) * G.keyl + p) * N + x];
    }
#pragma unroll
    for (int k = 0; k < BT; k++) {
      if (k < nct) {
        const u64 *dg = digits + (b0 + k) * dig_bs;
#pragma unroll
        for (int j = 0; j < BETA; j++) in.d[k][j] = dg[((size_t)j * G.pqn + r) * N + src];
        in.c0[k] = isq ? ct[(b0 + k) * ct_bs + (size_t)r * N + src] : 0;
      }
    }
#pragma unroll
    for (int gi = 0; gi < GT; gi++) {
      const int s = gi < ng ? BA.slot[i][gi] : -1;
      in.w[gi] = s >= 0 ? ptw(s) : 0;
    }
  };
  auto step = [&](const StepIn<GT, BT, BETA> &in) {
    typename M::Op w[GT], kb[BETA], ka[BETA];
#pragma unroll
    for (int gi = 0; gi < GT; gi++) w[gi] = M::prep(in.w[gi]);
#pragma unroll
    for (int j = 0; j < BETA; j++) {
      kb[j] = M::prep(in.kb[j]);
      ka[j] = M::prep(in.ka[j]);
    }
#pragma unroll
    for (int k = 0; k < BT; k++) {
      if (k < nct) {
        M ab, aa;
        ab.zero();
        aa.zero();
#pragma unroll
        for (int j = 0; j < BETA; j++) {
          const auto d = M::prep(in.d[k][j]);
          ab.mac(d, kb[j]);
          aa.mac(d, ka[j]);
        }
        u64 rb = ab.finish(pi.q, pi.qn);
        const auto RA = M::prep(aa.finish(pi.q, pi.qn));
        if (isq) rb = add_mod(rb, shoup(in.c0[k], pi.pmod, pi.pmod_p, pi.q), pi.q);
        const auto RB = M::prep(rb);
#pragma unroll
        for (int gi = 0; gi < GT; gi++) {
          acc[k][gi][0].mac(w[gi], RB);
          acc[k][gi][1].mac(w[gi], RA);
        }
      }
    }
  };
  StepIn<GT, BT, BETA> A, B;
  if (BA.nrot > 0) load(A, 0);
  for (int i = 0; i < BA.nrot; i += 2) {
    if (i + 1 < BA.nrot) load(B, i + 1);
    step(A);
    if (i + 1 >= BA.nrot) break;
    if (i + 2 < BA.nrot) load(A, i + 2);
    step(B);
  }
#pragma unroll
  for (int k = 0; k < BT; k++) {
    if (k >= nct) break;
    u64 *o = X + (b0 + k) * x_bs;
#pragma unroll
    for (int gi = 0; gi < GT; gi++) {
      if (gi < ng) {
        const size_t i0 = ((size_t)(gi * 2) * G.pqn + r) * N + x, i1 = ((size_t)(gi * 2 + 1) * G.pqn + r) * N + x;
        u64 v0 = acc[k][gi][0].finish(pi.q, pi.qn), v1 = acc[k][gi][1].finish(pi.q, pi.qn);
        if (accum) {
          v0 = add_mod(v0, o[i0], pi.q);
          v1 = add_mod(v1, o[i1], pi.q);
        }
        o[i0] = v0;
        o[i1] = v1;
      }
    }
  }
}

// One ciphertext and one giant output per thread: five waves per SIMD (at
// most 96 registers, a few of them spilled) measured faster than four.
template <int GT, int BT, int BETA, bool GEN>
__global__ __launch_bounds__(TPB, (GT * BT == 1 ? 5 : 1)) void baby_mac_kernel(
    BabyArgs BA, LevelGeom G, int L, int batch, int ntiles, const u64 *digits, size_t dig_bs, const u64 *ct,
    size_t ct_bs, const u64 *pt, size_t pt_words, int ng, u64 *X, size_t x_bs, int accum, const PrimeInfo *pinfo) {
  const int N = 1 << G.logn;
  const TileMap tm = chain_map(blockIdx.x, N / TPB, ntiles, G.pqn, G.limb_xcd, G.chain);
  const int x = tm.xb * TPB + threadIdx.x;
  const int p = pq_prime_dev(tm.r, G.level, L);
  const PrimeInfo pi = pinfo[p];
  if (pi.q < SPLIT_MAC_LIMIT)
    baby_mac_body<GT, BT, BETA, SplitMac, GEN>(BA, G, batch, x, tm.r, tm.tile * BT, p, pi, digits, dig_bs, ct,
                                               ct_bs, pt, pt_words, ng, X, x_bs, accum);
  else if (GEN && G.gen_wide)
    baby_mac_body<GT, BT, BETA, WideOf<GT * BT>, GEN>(BA, G, batch, x, tm.r, tm.tile * BT, p, pi, digits, dig_bs,
                                                      ct, ct_bs, pt, pt_words, ng, X, x_bs, accum);
  else
    baby_mac_body<GT, BT, BETA, WideOf<GT * BT>, false>(BA, G, batch, x, tm.r, tm.tile * BT, p, pi, digits,
                                                        dig_bs, ct, ct_bs, pt, pt_words, ng, X, x_bs, accum);
}

// The same product for launches with several giant outputs and a batch.  A
// workgroup of W wavefronts serves W ciphertexts on one 64-coefficient block
// of one limb.  Per baby step, wavefront w forms R_b of ciphertext w and puts
// it in LDS; then wavefront w multiplies its GPW giant outputs' plaintext
// words into R_b of all W ciphertexts.  Each plaintext word is read once per
// workgroup (W ciphertexts), each key word by W wavefronts of one CU at the
// same time (the repeats hit the CU's cache), and the accumulators spread
// over the workgroup: W * GPW * 2 per thread.  LDS holds R_b as the policy
// packs it (SplitMac: both 20-bit halves in one word).  The loads of the next
// rotation step are issued before the current step's barrier and products.
struct WidePack {
  static __device__ __forceinline__ u64 pack(u64 v) { return v; }
  static __device__ __forceinline__ u64 unpack(u64 v) { return v; }
};
struct SplitPack {
  static __device__ __forceinline__ u64 pack(u64 v) { return (v & 0xFFFFFull) | ((v >> 20) << 32); }
  static __device__ __forceinline__ Half20 unpack(u64 v) {
    Half20 h;
    h.lo = (uint32_t)v;
    h.hi = (uint32_t)(v >> 32);
    h.sum = h.lo + h.hi;
    return h;
  }
};
template <class M> struct PackOf;
template <> struct PackOf<WideMac> { using T = WidePack; };
template <> struct PackOf<SplitMac> { using T = SplitPack; };

template <int GPW, int BETA>
struct WaveIn {
  u64 kb[BETA], ka[BETA], d[BETA], c0, w[GPW];
};

template <int W, int GPW, int BETA, class M>
__device__ __forceinline__ void baby_shared_body(u64 (*R)[W][2][64], const BabyArgs &BA, const LevelGeom &G,
                                                 int batch, int x, int lane, int w, int r, int b0, int p,
                                                 const PrimeInfo &pi, const u64 *digits, size_t dig_bs,
                                                 const u64 *ct, size_t ct_bs, const u64 *pt, int ng, u64 *X,
                                                 size_t x_bs, int accum) {
  using Pk = typename PackOf<M>::T;
  const int N = 1 << G.logn;
  const int nct = min(W, batch - b0);
  const bool isq = r <= G.level;
  const bool mine = w < nct;                // this wavefront forms R_b of ciphertext b0 + w
  const int gw = w * GPW;                   // its first giant output (relative to g0)
  const u64 *c = ct + (b0 + (mine ? w : 0)) * ct_bs;
  const u64 *dg = digits + (b0 + (mine ? w : 0)) * dig_bs;
  M acc[W][GPW][2];
#pragma unroll
  for (int k = 0; k < W; k++)
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) {
      acc[k][gi][0].zero();
      acc[k][gi][1].zero();
    }
  auto macs = [&](u64 (*Rb)[2][64], const u64 *wraw) {
    typename M::Op wv[GPW];
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) wv[gi] = M::prep(wraw[gi]);
#pragma unroll
    for (int k = 0; k < W; k++) {
      if (k < nct) {
        const auto RB = Pk::unpack(Rb[k][0][lane]);
        const auto RA = Pk::unpack(Rb[k][1][lane]);
#pragma unroll
        for (int gi = 0; gi < GPW; gi++) {
          acc[k][gi][0].mac(wv[gi], RB);
          acc[k][gi][1].mac(wv[gi], RA);
        }
      }
    }
  };
  int buf = 0;
  if (BA.has0 && isq) {   // R_0 = P (c0, c1); it vanishes on the special limbs
    u64 w0[GPW];
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) {
      const int s = gw + gi < ng ? BA.slot0[gw + gi] : -1;
      w0[gi] = s >= 0 ? pt[((size_t)s * G.pqn + r) * N + x] : 0;
    }
    if (mine) {
      R[0][w][0][lane] = Pk::pack(shoup(c[(size_t)r * N + x], pi.pmod, pi.pmod_p, pi.q));
      R[0][w][1][lane] = Pk::pack(shoup(c[((size_t)(G.level + 1) + r) * N + x], pi.pmod, pi.pmod_p, pi.q));
    }
    __syncthreads();
    macs(R[0], w0);
    buf = 1;
  }
  // One set of registers per wavefront for the step inputs: the key, digit
  // and c0 words of step i+1 are requested as soon as R_b of step i is in
  // LDS, the plaintext words of step i+1 as soon as those of step i are
  // converted, so both loads overlap the barrier and products of step i.
  WaveIn<GPW, BETA> in;
  auto load_r = [&](int i) {
    if (mine) {
      const unsigned src = galois_src(x, BA.gal[i], G.logn);
      const u64 *kk = BA.key[i];
#pragma unroll
      for (int j = 0; j < BETA; j++) {
        in.kb[j] = kk[((size_t)(2 * j) * G.keyl + p) * N + x];
        in.ka[j] = kk[((size_t)(2 * j + 1) * G.keyl + p) * N + x];
        in.d[j] = dg[((size_t)j * G.pqn + r) * N + src];
      }
      in.c0 = isq ? c[(size_t)r * N + src] : 0;
    }
  };
  auto load_w = [&](int i) {
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) {
      const int s = gw + gi < ng ? BA.slot[i][gw + gi] : -1;
      in.w[gi] = s >= 0 ? pt[((size_t)s * G.pqn + r) * N + x] : 0;
    }
  };
  if (BA.nrot > 0) {
    load_r(0);
    load_w(0);
  }
  for (int i = 0; i < BA.nrot; i++) {
    if (mine) {
      M ab, aa;
      ab.zero();
      aa.zero();
#pragma unroll
      for (int j = 0; j < BETA; j++) {
        const auto d = M::prep(in.d[j]);
        ab.mac(d, M::prep(in.kb[j]));
        aa.mac(d, M::prep(in.ka[j]));
      }
      u64 RB = ab.finish(pi.q, pi.qn);
      const u64 RA = aa.finish(pi.q, pi.qn);
      if (isq) RB = add_mod(RB, shoup(in.c0, pi.pmod, pi.pmod_p, pi.q), pi.q);
      R[buf][w][0][lane] = Pk::pack(RB);
      R[buf][w][1][lane] = Pk::pack(RA);
    }
    if (i + 1 < BA.nrot) load_r(i + 1);
    __syncthreads();
    typename M::Op wv[GPW];
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) wv[gi] = M::prep(in.w[gi]);
    if (i + 1 < BA.nrot) load_w(i + 1);
#pragma unroll
    for (int k = 0; k < W; k++) {
      if (k < nct) {
        const auto RB = Pk::unpack(R[buf][k][0][lane]);
        const auto RA = Pk::unpack(R[buf][k][1][lane]);
#pragma unroll
        for (int gi = 0; gi < GPW; gi++) {
          acc[k][gi][0].mac(wv[gi], RB);
          acc[k][gi][1].mac(wv[gi], RA);
        }
      }
    }
    // the next step writes the other buffer; the one after that comes only
    // after the next barrier, which every wavefront passes once done here
    buf ^= 1;
  }
#pragma unroll
  for (int k = 0; k < W; k++) {
    if (k >= nct) break;
    u64 *o = X + (b0 + k) * x_bs;
#pragma unroll
    for (int gi = 0; gi < GPW; gi++) {
      const int g = gw + gi;
      if (g < ng) {
        const size_t i0 = ((size_t)(g * 2) * G.pqn + r) * N + x, i1 = ((size_t)(g * 2 + 1) * G.pqn + r) * N + x;
        u64 v0 = acc[k][gi][0].finish(pi.q, pi.qn), v1 = acc[k][gi][1].finish(pi.q, pi.qn);
        if (accum) {
          v0 = add_mod(v0, o[i0], pi.q);
          v1 = add_mod(v1, o[i1], pi.q);
        }
        o[i0] = v0;
        o[i1] = v1;
      }
    }
  }
}

template <int W, int GPW, int BETA>
__global__ __launch_bounds__(64 * W) void baby_mac_shared_kernel(BabyArgs BA, LevelGeom G, int L, int batch,
                                                                 int ntiles, const u64 *digits, size_t dig_bs,
                                                                 const u64 *ct, size_t ct_bs, const u64 *pt,
                                                                 int ng, u64 *X, size_t x_bs, int accum,
                                                                 const PrimeInfo *pinfo) {
  __shared__ u64 R[2][W][2][64];
  const int N = 1 << G.logn;
  const TileMap tm = chain_map(blockIdx.x, N / 64, ntiles, G.pqn, G.limb_xcd, G.chain);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int x = tm.xb * 64 + lane;
  const int p = pq_prime_dev(tm.r, G.level, L);
  const PrimeInfo pi = pinfo[p];
  if (pi.q < SPLIT_MAC_LIMIT)
    baby_shared_body<W, GPW, BETA, SplitMac>(R, BA, G, batch, x, lane, w, tm.r, tm.tile * W, p, pi, digits,
                                             dig_bs, ct, ct_bs, pt, ng, X, x_bs, accum);
  else
    baby_shared_body<W, GPW, BETA, WideMac>(R, BA, G, batch, x, lane, w, tm.r, tm.tile * W, p, pi, digits,
                                            dig_bs, ct, ct_bs, pt, ng, X, x_bs, accum);
}

// ---------------------------------------------------------------- matrix-core plaintext MAC
//
// For a batch, the plaintext MAC of the baby-step stage is a dense integer
// contraction at every coefficient x of every limb:
//   X_g[c] = sum_b pt_{g,b}[x] R_b[c][x]     (both polynomials of every c),
// rows (ciphertext, polynomial), columns the giant outputs, depth the baby
// steps.  It runs on the int8 matrix cores exactly: a residue v in [0, q) is
// centred to (-q/2, q/2) and written with P balanced base-256 digits d_i in
// [-128, 127] (P = 5 below 2^40, 8 otherwise), v = sum_i d_i 256^i; the bytes
// of (v + OFF) xor OFF, OFF = 0x80 repeated P times, are exactly those digits.
// Then sum_b pt R = sum_s 256^s sum_{i+j=s} sum_b pt_j R_i, and every inner
// sum over the (at most 64) baby steps is one v_mfma_i32_16x16x64_i8 product
// (|partial| < 2^22).  The columns are rebuilt into the exact signed 128-bit
// sum and reduced with one Montgomery reduction (the plaintexts are in
// Montgomery form), which gives the same canonical residue as the VALU kernels.
//
// Operand layouts (16x16x64, lane l = 16 h + n): A holds row n, depths
// 16 h .. 16 h + 15 in its 16 bytes; B holds column n, the same depths; the
// result holds column n, rows 4 h .. 4 h + 3.  A row is (ciphertext,
// polynomial) = (n / 2, n % 2) of 8 ciphertexts; a column n is giant n % 8
// and digit 2 jp + n / 8 of the plaintext word (two digits of B per product),
// so result tile s = i + 2 jp holds the column sums s (n < 8) and s + 1
// (n >= 8), which lanes n and n ^ 8 exchange.

typedef int v4i __attribute__((ext_vector_type(4)));

template <int P>
struct Balanced {
  static constexpr u64 OFF = P == 8 ? 0x8080808080808080ull : 0x8080808080ull;
  // P digits hold [-OFF, 256^P - OFF): for q near 2^40 that is narrower than
  // (-q/2, q/2], so the values from min((q + 1) / 2, 256^P - OFF) on are
  // taken as v - q (which is >= -OFF since q <= 256^P)
  static constexpr u64 LIM = P == 8 ? 0x7F7F7F7F7F7F7F80ull : 0x7F7F7F7F80ull;
  // v in [0, q) -> the P digit bytes of its signed representative
  static __device__ __forceinline__ u64 of(u64 v, u64 q) {
    const u64 thr = min((q + 1) >> 1, LIM);
    const u64 c = v >= thr ? v - q : v;   // two's complement of the signed value
    return (c + OFF) ^ OFF;
  }
};

// Bytes p of four words, packed in order into one 32-bit word.
__device__ __forceinline__ uint32_t byte_quad(u64 a, u64 b, u64 c, u64 d, int p) {
  const int sh = 8 * (p & 3);
  const uint32_t wa = (uint32_t)(p < 4 ? a : a >> 32), wb = (uint32_t)(p < 4 ? b : b >> 32);
  const uint32_t wc = (uint32_t)(p < 4 ? c : c >> 32), wd = (uint32_t)(p < 4 ? d : d >> 32);
  return ((wa >> sh) & 0xFFu) | (((wb >> sh) & 0xFFu) << 8) | (((wc >> sh) & 0xFFu) << 16) |
         (((wd >> sh) & 0xFFu) << 24);
}

// Limbs of one matrix-core launch (those of one digit count P).
struct LimbSel {
  int n;
  unsigned char r[HELRM_MAX_LIMBS];
};

constexpr int MF_XB = 8;    // coefficients per workgroup (one per wavefront in the products)
constexpr int MF_CT = 8;    // ciphertexts per workgroup (16 rows)
constexpr int MF_TPB = 512;

// R_b of ciphertext c at coefficient x (both polynomials, canonical), for
// depth index k of the launch: k = 0 is b = 0 when has0, then the rotations.
template <int BETA, class M>
__device__ __forceinline__ void form_r(const BabyArgs &BA, const LevelGeom &G, int k, int x, int r, int p,
                                      const PrimeInfo &pi, const u64 *dg, const u64 *c, bool isq, u64 &RB,
                                      u64 &RA) {
  const int N = 1 << G.logn;
  RB = RA = 0;
  if (BA.has0 && k == 0) {
    if (isq) {
      RB = shoup(c[(size_t)r * N + x], pi.pmod, pi.pmod_p, pi.q);
      RA = shoup(c[((size_t)(G.level + 1) + r) * N + x], pi.pmod, pi.pmod_p, pi.q);
    }
    return;
  }
  const int i = k - BA.has0;
  if (i < 0 || i >= BA.nrot) return;
  const unsigned src = galois_src(x, BA.gal[i], G.logn);
  const u64 *kk = BA.key[i];
  M ab, aa;
  ab.zero();
  aa.zero();
#pragma unroll
  for (int j = 0; j < BETA; j++) {
    const auto d = M::prep(dg[((size_t)j * G.pqn + r) * N + src]);
    ab.mac(d, M::prep(kk[((size_t)(2 * j) * G.keyl + p) * N + x]));
    aa.mac(d, M::prep(kk[((size_t)(2 * j + 1) * G.keyl + p) * N + x]));
  }
  RB = ab.finish(pi.q, pi.qn);
  RA = aa.finish(pi.q, pi.qn);
  if (isq) RB = add_mod(RB, shoup(c[(size_t)r * N + src], pi.pmod, pi.pmod_p, pi.q), pi.q);
}

template <int BETA, int P, class M>
__device__ __forceinline__ void baby_mfma_body(uint32_t *A, u64 *O, const BabyArgs &BA, const LevelGeom &G,
                                               int batch, int xb, int r, int b0, int p, const PrimeInfo &pi,
                                               const u64 *digits, size_t dig_bs, const u64 *ct, size_t ct_bs,
                                               const uint8_t *ptm, int ng, u64 *X, size_t x_bs, int accum) {
  constexpr int NJP = (P + 1) / 2;          // B operands: two digits each
  constexpr int NS = P + 2 * (NJP - 1);     // result tiles s = i + 2 jp
  const int N = 1 << G.logn;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const bool isq = r <= G.level;
  // the plaintext operands of this wavefront's coefficient, in flight during step 1
  v4i bop[NJP];
  {
    const uint8_t *bp = ptm + (((size_t)r * N + xb * MF_XB + w) * 4) * 1024 + lane * 16;
#pragma unroll
    for (int jp = 0; jp < NJP; jp++) bop[jp] = *(const v4i *)(bp + jp * 1024);
  }
  // 1. R_b for (coefficient xi, ciphertext ci, depths 8 w .. 8 w + 7), as
  //    balanced digits into A[xi][digit][row][depth]
  {
    const int xi = t & 7, ci = (t >> 3) & 7, x = xb * MF_XB + xi, c = b0 + ci;
    const bool ok = c < batch;
    const u64 *dg = digits + (size_t)(ok ? c : b0) * dig_bs;
    const u64 *cc = ct + (size_t)(ok ? c : b0) * ct_bs;
#pragma unroll 1
    for (int kq = 0; kq < 2; kq++) {
      u64 rb[4], ra[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        rb[u] = ra[u] = 0;
        if (ok) form_r<BETA, M>(BA, G, 8 * w + 4 * kq + u, x, r, p, pi, dg, cc, isq, rb[u], ra[u]);
        rb[u] = Balanced<P>::of(rb[u], pi.q);
        ra[u] = Balanced<P>::of(ra[u], pi.q);
      }
#pragma unroll
      for (int d = 0; d < P; d++) {
        uint32_t *row = A + ((xi * P + d) * 16 + 2 * ci) * 16 + 2 * w + kq;
        row[0] = byte_quad(rb[0], rb[1], rb[2], rb[3], d);
        row[16] = byte_quad(ra[0], ra[1], ra[2], ra[3], d);
      }
    }
  }
  __syncthreads();
  // 2. coefficient xi = w: P x NJP products, column sums, exact sum, REDC
  const int n = lane & 15, h = lane >> 4, hf = n >> 3, g = n & 7;
  u64 res[2];
  {
    const int xi = w;
    v4i acc[NS];
#pragma unroll
    for (int k = 0; k < NS; k++) acc[k] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < P; i++) {
      const v4i aop = *(const v4i *)(A + ((xi * P + i) * 16 + n) * 16 + 4 * h);
#pragma unroll
      for (int jp = 0; jp < NJP; jp++)
        acc[i + 2 * jp] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, bop[jp], acc[i + 2 * jp], 0, 0, 0);
    }
    // lanes n and n ^ 8 hold the two digit halves of one giant's column sums
    // (tile s: column s for n < 8, column s + 1 for n >= 8).  Each lane
    // finishes two rows (2 hf + vv): column c = own tile c (n < 8) or c - 1
    // (n >= 8) plus what lane n ^ 8 sends for that row.
#pragma unroll
    for (int vv = 0; vv < 2; vv++) {
      u128 S = 0;   // the exact signed sum (|S| < 2^126) in two's complement mod 2^128
#pragma unroll
      for (int cidx = 0; cidx <= NS; cidx++) {
        const int lo_t = cidx < NS ? acc[cidx][vv] : 0, lo_o = cidx < NS ? acc[cidx][2 + vv] : 0;
        const int up_t = cidx >= 1 ? acc[cidx - 1][vv] : 0, up_o = cidx >= 1 ? acc[cidx - 1][2 + vv] : 0;
        // n < 8: own tile c at row vv, partner's tile c - 1 at row vv;
        // n >= 8: own tile c - 1 at row 2 + vv, partner's tile c at row 2 + vv
        const int own = hf ? up_o : lo_t;
        const int send = hf ? up_t : lo_o;
        const long long col = (long long)own + (long long)__shfl_xor(send, 8);
        S += (u128)(__int128)col << (8 * cidx);
      }
      long long hi = (long long)(u64)(S >> 64);
      const u64 lo = (u64)S;
      const long long q = (long long)pi.q;
      if (hi < 0) hi += q;
      if (hi < 0) hi += q;
      if (hi >= q) hi -= q;
      res[vv] = redc(lo, (u64)hi, pi.q, pi.qn);
    }
  }
  __syncthreads();   // every wave is done with A: its space stages the results
#pragma unroll
  for (int vv = 0; vv < 2; vv++) O[(w * 16 + 4 * h + 2 * hf + vv) * 8 + g] = res[vv];
  __syncthreads();
  // 3. results: runs of 8 coefficients per (ciphertext, giant, polynomial)
  {
    const int xi = t & 7, gg = (t >> 3) & 7, rq = t >> 6, x = xb * MF_XB + xi;
    if (gg < ng) {
#pragma unroll
      for (int k = 0; k < 2; k++) {
        const int row = 2 * rq + k, c = b0 + (row >> 1), pol = row & 1;
        if (c >= batch) continue;
        u64 v = O[(xi * 16 + row) * 8 + gg];
        u64 *o = X + (size_t)c * x_bs + ((size_t)(gg * 2 + pol) * G.pqn + r) * N + x;
        if (accum) v = add_mod(v, *o, pi.q);
        *o = v;
      }
    }
  }
}

template <int BETA, int P>
__global__ __launch_bounds__(MF_TPB, 4) void baby_mfma_kernel(BabyArgs BA, LevelGeom G, int L, int batch,
                                                               int ntiles, LimbSel ls, const u64 *digits,
                                                               size_t dig_bs, const u64 *ct, size_t ct_bs,
                                                               const uint8_t *ptm, int ng, u64 *X, size_t x_bs,
                                                               int accum, const PrimeInfo *pinfo,
                                                               const u64 *chain) {
  __shared__ __align__(16) uint32_t A[MF_XB * P * 16 * 16];
  static_assert(MF_XB * P * 16 * 16 * 4 >= MF_XB * 16 * 8 * 8, "result staging fits in A");
  const int N = 1 << G.logn;
  const TileMap tm = chain_map(blockIdx.x, N / MF_XB, ntiles, ls.n, G.limb_xcd, chain);
  const int r = ls.r[tm.r];
  const int p = pq_prime_dev(r, G.level, L);
  const PrimeInfo pi = pinfo[p];
  if (P == 5)
    baby_mfma_body<BETA, P, SplitMac>(A, (u64 *)A, BA, G, batch, tm.xb, r, tm.tile * MF_CT, p, pi, digits, dig_bs,
                                      ct, ct_bs, ptm, ng, X, x_bs, accum);
  else
    baby_mfma_body<BETA, P, WideMac>(A, (u64 *)A, BA, G, batch, tm.xb, r, tm.tile * MF_CT, p, pi, digits, dig_bs,
                                     ct, ct_bs, ptm, ng, X, x_bs, accum);
}

// ---------------------------------------------------------------- key-folded matrix-core product
//
// With the keys folded into the plaintexts the whole baby-step stage of a
// batch is one integer contraction per coefficient and limb:
//   X_g[c] = sum_b pt_{g,b} R_b[c],  R_b = sum_j sigma_b(d_j) k_{b,j} (+ P sigma_b(c0))
//          = sum_{b,e} sigma_b(y_e[c]) W_{g,b,e},   W_{g,b,e} = pt_{g,b} k_{b,e}
// with y_e the digits d_0..d_{beta'-1} and c0 (whose "key" is P, on the Q
// limbs), and for b = 0 the unrotated c0 and c1 with W = pt_{g,0} P on the
// polynomial they feed: the same residues mod q (the sum is only
// reassociated), with no per-rotation key switch left to form.  Rows are the
// ciphertexts (16 per product), columns (giant, polynomial) (16), depth the
// (baby step, entry) pairs, 4 entries per baby step (beta' <= 3; unused
// entries are zero), in chunks of 64; the operands are balanced base-256
// digits as in the MAC above, here P x P products per chunk (tile s = i + j
// holds column s), rebuilt into the exact sum and reduced once.  The folded
// words are built once per plan and key set (wfold_pack_kernel, 1 KiB per
// digit, chunk, limb, coefficient and giant tile).

struct FoldRun {
  int nslot, has0, kc;                 // baby slots (b = 0 first when has0), depth chunks of 64
  unsigned gal[HELRM_MAX_BABY];        // Galois element of rotation slot has0 + i
  unsigned off[HELRM_MAX_PRIMES];      // limb r's block in the tile, in units of N * kc KiB
};

constexpr int FD_RS = 20;             // LDS dwords per ciphertext row (16 used): conflict-free 16-byte accesses

template <int P>
struct FoldLds {
  static constexpr int PS = 16 * FD_RS;        // dwords per digit plane (16 ciphertexts)
  // dwords per coefficient: 4 mod 32, so the 8 coefficients that one
  // 16-byte store instruction's lanes write land in 8 distinct bank groups
  static constexpr int XS = P * PS + 4;
  static constexpr int WORDS = MF_XB * XS;
  static constexpr int OS = 16 * 16 + 2;       // result staging: u64 per coefficient (2 mod 16)
};

// One workgroup: coefficient block xb (8 coefficients, one per wave) of limb
// r, row tiles [mt_begin, mt_end) of 16 ciphertexts in groups of MP, each
// group over FR.kc depth chunks; a chunk's folded operands are loaded once
// and serve the MP tiles of the group (MP x (2P - 1) accumulator tiles).
// The sub-steps (group, chunk, tile) are software-pipelined: the gathers of
// the next sub-step's entries are issued before this one's barrier and
// products, the next chunk's folded operands right after the products of a
// chunk's last tile, so their latency overlaps the matrix-core work.
template <int P, int MP>
__device__ __forceinline__ void baby_fold_body(uint32_t *A, const unsigned *sgal, const FoldRun &FR,
                                               const LevelGeom &G, int batch, int xb, int r, const PrimeInfo &pi,
                                               const uint32_t *E, size_t e_bs, size_t e_half, const uint8_t *wm, int ng,
                                               u64 *X, size_t x_bs, int accum, int mt_begin, int mt_end) {
  using LD = FoldLds<P>;
  constexpr int NS = 2 * P - 1;
  const int N = 1 << G.logn;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int n = lane & 15, h = lane >> 4;
  const uint8_t *wx = wm + ((size_t)FR.off[r] * N * FR.kc + (size_t)(xb * MF_XB + w) * FR.kc * P) * 1024 + lane * 16;
  const int K = FR.kc, groups = (mt_end - mt_begin + MP - 1) / MP;
  if (groups <= 0) return;
  // staging role of this thread: coefficient xi, ciphertext ci of the tile,
  // slots 16 kc + 4 sq .. + 3
  const int sxi = t & 7, sci = (t >> 3) & 15, sq = t >> 7, sx = xb * MF_XB + sxi;
  const uint32_t *elimb = E + (size_t)FR.off[r] * N;
  uint32_t q4[P][4];
  unsigned qmask = 0;   // slots of the gathered sub-step that hold entries (the others stage as 0)
  // the entries of tile mt, chunk kc: balanced digits packed per digit plane
  // by fold_entries_kernel, gathered at the rotation's source.  Branch-free:
  // an absent ciphertext (a tile past the batch included) or slot loads valid
  // words of ciphertext 0 / coefficient x and is masked out when staged, so
  // the loads stay in flight across the barrier and the products that follow
  auto gather = [&](int mt, int kc) {
    const int c = mt * 16 + sci;
    const bool ok = c < batch;
    const uint32_t *ec = elimb + (size_t)(ok ? c : 0) * e_bs;
    qmask = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int sl = 16 * kc + 4 * sq + u;
      const bool zero = FR.has0 && sl == 0;
      const int gi = min(max(sl - FR.has0, 0), FR.nslot - FR.has0 - 1);
      const unsigned src = zero || gi < 0 ? (unsigned)sx : galois_src(sx, sgal[gi < 0 ? 0 : gi], G.logn);
      const uint32_t *ep = ec + (zero ? e_half : 0) + (size_t)src * P;
#pragma unroll
      for (int d = 0; d < P; d++) q4[d][u] = ep[d];
      qmask |= (ok && sl < FR.nslot) ? 1u << u : 0u;
    }
  };
  v4i wop[P];
  auto load_w = [&](int kc) {
#pragma unroll
    for (int j = 0; j < P; j++) wop[j] = *(const v4i *)(wx + ((size_t)kc * P + j) * 1024);
  };
  v4i acc[MP][NS];
#pragma unroll
  for (int m = 0; m < MP; m++)
#pragma unroll
    for (int k = 0; k < NS; k++) acc[m][k] = v4i{0, 0, 0, 0};
  load_w(0);
  gather(mt_begin, 0);
  for (int g = 0; g < groups; g++) {
    const int mt0 = mt_begin + g * MP;
    for (int kc = 0; kc < K; kc++) {
#pragma unroll
      for (int m = 0; m < MP; m++) {
#pragma unroll
        for (int d = 0; d < P; d++)
          *(v4i *)(A + sxi * LD::XS + d * LD::PS + sci * FD_RS + 4 * sq) =
              v4i{(int)(qmask & 1 ? q4[d][0] : 0u), (int)(qmask & 2 ? q4[d][1] : 0u),
                  (int)(qmask & 4 ? q4[d][2] : 0u), (int)(qmask & 8 ? q4[d][3] : 0u)};
        // the next sub-step's entries (unconditional: the last re-reads its
        // own), so every sub-step issues the same loads
        {
          int nm = mt0 + m + 1, nk = kc;
          if (m + 1 == MP) {
            nm = mt0;
            nk = kc + 1;
            if (nk == K) {
              nk = 0;
              nm = g + 1 < groups ? mt0 + MP : mt0 + m;
              if (g + 1 == groups) nk = kc;
            }
          }
          gather(nm, nk);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < P; i++) {
          const v4i aop = *(const v4i *)(A + w * LD::XS + i * LD::PS + n * FD_RS + 4 * h);
#pragma unroll
          for (int j = 0; j < P; j++)
            acc[m][i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop, wop[j], acc[m][i + j], 0, 0, 0);
        }
        if (m + 1 == MP) load_w(kc + 1 < K ? kc + 1 : 0);
        __syncthreads();
      }
    }
    // group done: lane holds rows (ciphertexts) 4 h + v of column n = (giant
    // n % 8, polynomial n / 8) of every tile of the group
#pragma unroll
    for (int m = 0; m < MP; m++) {
      const int mt = mt0 + m;
      u64 res[4];
#pragma unroll
      for (int v = 0; v < 4; v++) {
        u128 S = 0;   // the exact signed sum in two's complement mod 2^128
#pragma unroll
        for (int cidx = 0; cidx < NS; cidx++) S += (u128)(__int128)(long long)acc[m][cidx][v] << (8 * cidx);
        const long long hi = (long long)(u64)(S >> 64);
        const u64 lo = (u64)S;
        // |S| < 2^87 (P = 5) or 2^127 (P = 8): |hi| < 2^23, or below 8 q (q > 2^59)
        u64 hm;
        if (P == 5)
          hm = hi < 0 ? (u64)(hi + (long long)pi.q) : (u64)hi;
        else
          hm = reduce64((u64)(hi + 8 * (long long)pi.q), pi.q, pi.mu);
        res[v] = redc(lo, hm, pi.q, pi.qn);
      }
#pragma unroll
      for (int k = 0; k < NS; k++) acc[m][k] = v4i{0, 0, 0, 0};
      u64 *O = (u64 *)A;   // the staging area is free: every wave passed the last barrier
#pragma unroll
      for (int v = 0; v < 4; v++) O[w * LD::OS + (4 * h + v) * 16 + n] = res[v];
      __syncthreads();
      {
        const int xi = t & 7, col = (t >> 3) & 15, rq = t >> 7, x = xb * MF_XB + xi;
        const int gg = col & 7, pol = col >> 3;
        if (gg < ng) {
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int row = 4 * rq + k, c = mt * 16 + row;
            if (c >= batch) continue;
            u64 v = O[xi * LD::OS + row * 16 + col];
            u64 *o = X + (size_t)c * x_bs + ((size_t)(gg * 2 + pol) * G.pqn + r) * N + x;
            if (accum) v = add_mod(v, *o, pi.q);
            *o = v;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int P, int MP>
__global__ __launch_bounds__(MF_TPB, MP == 1 ? 2 : 1) void baby_fold_kernel(FoldRun FR, LevelGeom G, int L,
                                                                             int batch, LimbSel ls,
                                                                             const uint32_t *E, size_t e_bs,
                                                                             size_t e_half, const uint8_t *wm,
                                                                             int ng, u64 *X, size_t x_bs, int accum,
                                                                             const PrimeInfo *pinfo,
                                                                             const u64 *chain) {
  __shared__ __align__(16) uint32_t A[FoldLds<P>::WORDS];
  __shared__ unsigned sgal[HELRM_MAX_BABY];   // the rotations' Galois elements, read with LDS latency
  static_assert(FoldLds<P>::WORDS * 4 >= MF_XB * FoldLds<P>::OS * 8, "result staging fits");
  const int N = 1 << G.logn;
  if (threadIdx.x < HELRM_MAX_BABY) sgal[threadIdx.x] = FR.gal[threadIdx.x];
  __syncthreads();
  const TileMap tm = chain_map(blockIdx.x, N / MF_XB, 1, ls.n, G.limb_xcd, chain);
  const int r = ls.r[tm.r];
  const PrimeInfo pi = pinfo[pq_prime_dev(r, G.level, L)];
  // one workgroup takes every row tile of its coefficient block
  baby_fold_body<P, MP>(A, sgal, FR, G, batch, tm.xb, r, pi, E, e_bs, e_half, wm, ng, X, x_bs, accum, 0,
                        (batch + 15) / 16);
}

// The entries of every ciphertext once, before the folded product gathers
// them per rotation: at limb r and coefficient x, P words whose bytes are
// digit d of (d_0, .., d_{beta'-1}, c0, 0..) (E, the rotated steps; c0 on the
// Q limbs only) and of (c0, c1, 0, 0) (E + e_half, step b = 0; Q limbs only),
// limb r's words starting at off[r] N.
template <int BETA>
__global__ __launch_bounds__(256) void fold_entries_kernel(const u64 *digits, size_t dig_bs, const u64 *ct,
                                                           size_t ct_bs, uint32_t *E, size_t e_bs, size_t e_half,
                                                           FoldRun FR, LevelGeom G, int L, const PrimeInfo *pinfo) {
  const int N = 1 << G.logn;
  const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;   // r N + x
  const int c = blockIdx.y, x = (int)(tid % N), r = (int)(tid / N);
  if (r >= G.pqn) return;
  const PrimeInfo pi = pinfo[pq_prime_dev(r, G.level, L)];
  const bool isq = r <= G.level, wide = pi.q >= SPLIT_MAC_LIMIT;
  const u64 *dg = digits + (size_t)c * dig_bs;
  const u64 *cc = ct + (size_t)c * ct_bs;
  u64 e[4] = {0, 0, 0, 0}, z[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < BETA; j++) e[j] = dg[((size_t)j * G.pqn + r) * N + x];
  if (isq) {
    e[BETA] = z[0] = cc[(size_t)r * N + x];
    z[1] = cc[((size_t)(G.level + 1) + r) * N + x];
  }
  uint32_t *o = E + (size_t)c * e_bs + (size_t)FR.off[r] * N;
  if (wide) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      e[j] = Balanced<8>::of(e[j], pi.q);
      z[j] = Balanced<8>::of(z[j], pi.q);
    }
#pragma unroll
    for (int d = 0; d < 8; d++) {
      o[(size_t)x * 8 + d] = byte_quad(e[0], e[1], e[2], e[3], d);
      o[e_half + (size_t)x * 8 + d] = byte_quad(z[0], z[1], z[2], z[3], d);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      e[j] = Balanced<5>::of(e[j], pi.q);
      z[j] = Balanced<5>::of(z[j], pi.q);
    }
#pragma unroll
    for (int d = 0; d < 5; d++) {
      o[(size_t)x * 5 + d] = byte_quad(e[0], e[1], e[2], e[3], d);
      o[e_half + (size_t)x * 5 + d] = byte_quad(z[0], z[1], z[2], z[3], d);
    }
  }
}

// Folded operands of one giant tile: thread (r, x, chunk, digit, lane)
// writes the 16 bytes of lane l = 16 h + n: digit `d` of W for column n
// (giant n % 8, polynomial n / 8) at depths 64 kc + 16 h .. + 15, depth k =
// 4 slot + entry.  W = REDC(pt_mont k_mont) (Montgomery form of pt k) for the
// digit entries, pt_mont P for the c0 entry (Q limbs), and for slot 0 with
// b = 0, pt_mont P on c0 (polynomial 0) and c1 (polynomial 1).
struct FoldPack {
  int nslot, has0, kc, beta, ng;
  const u64 *key[HELRM_MAX_BABY];
  short slot[HELRM_MAX_BABY + 1][8];   // stored diagonal of (slot, giant), -1: none
  unsigned off[HELRM_MAX_PRIMES];
  unsigned char planes[HELRM_MAX_PRIMES];
};

__global__ __launch_bounds__(256) void wfold_pack_kernel(const FoldPack FP, const u64 *pt, uint8_t *wm, int pqn,
                                                         int level, int L, int logn, int keyl,
                                                         const PrimeInfo *pinfo) {
  const int N = 1 << logn;
  // x: ((r N + x) 8 + d) 64 + l; y: the depth chunk (a grid holds fewer than 2^32 work-items per dimension)
  const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int l = tid & 63, d = (tid >> 6) & 7;
  const int kci = blockIdx.y;
  const size_t rx = tid >> 9;
  const int x = (int)(rx % N), r = (int)(rx / N);
  if (r >= pqn) return;
  const int P = FP.planes[r];
  if (d >= P) return;
  const int p = pq_prime_dev(r, level, L);
  const PrimeInfo pi = pinfo[p];
  const bool isq = r <= level;
  const int n = l & 15, h = l >> 4, g = n & 7, pol = n >> 3;
  uint32_t wv[4] = {0, 0, 0, 0};
  for (int tt = 0; tt < 16; tt++) {
    const int k = 64 * kci + 16 * h + tt, sl = k >> 2, e = k & 3;
    if (sl >= FP.nslot || g >= FP.ng) continue;
    const int di = FP.slot[sl][g];
    if (di < 0) continue;
    const u64 ptm = pt[((size_t)di * pqn + r) * N + x];
    u64 v = 0;
    if (FP.has0 && sl == 0) {
      if (isq && e == pol) v = shoup(ptm, pi.pmod, pi.pmod_p, pi.q);
    } else if (e < FP.beta) {
      const u64 kw = FP.key[sl - FP.has0][((size_t)(2 * e + pol) * keyl + p) * N + x];
      const u128 prod = (u128)ptm * kw;
      v = redc((u64)prod, (u64)(prod >> 64), pi.q, pi.qn);
    } else if (e == FP.beta) {
      if (isq && pol == 0) v = shoup(ptm, pi.pmod, pi.pmod_p, pi.q);
    }
    const u64 bal = P == 5 ? Balanced<5>::of(v, pi.q) : Balanced<8>::of(v, pi.q);
    wv[tt >> 2] |= (uint32_t)((bal >> (8 * d)) & 0xFFu) << (8 * (tt & 3));
  }
  uint32_t *o = (uint32_t *)(wm + (((size_t)FP.off[r] * N * FP.kc + ((size_t)x * FP.kc + kci) * P + d) * 1024) + l * 16);
  o[0] = wv[0];
  o[1] = wv[1];
  o[2] = wv[2];
  o[3] = wv[3];
}

// B operands of the matrix-core MAC, built once per plan: for giant tile T,
// limb r, coefficient x and digit pair jp, 64 lanes x 16 bytes where lane
// l = 16 h + n holds the balanced digit 2 jp + n / 8 of pt_{8T + n % 8, b}[x]
// for the depths k = 16 h .. 16 h + 15 (b = the k-th baby step of the tile,
// slot_tab[T][k][g] gives its stored diagonal, -1 none).  4 KiB per (T, r, x).
__global__ __launch_bounds__(256) void ptm_pack_kernel(const u64 *pt, const int *slot_tab, uint8_t *ptm, int pqn,
                                                       int level, int L, int N, const PrimeInfo *pinfo) {
  // x: (r N + x) 256 + jp 64 + l; y: the giant tile T
  const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int l = tid & 63, jp = (tid >> 6) & 3;
  const int T = blockIdx.y;
  const size_t trx = (size_t)T * pqn * N + (tid >> 8);
  const int x = (int)(trx % N), r = (int)((trx / N) % pqn);
  const PrimeInfo pi = pinfo[pq_prime_dev(r, level, L)];
  const int P = pi.q < SPLIT_MAC_LIMIT ? 5 : 8;
  const int n = l & 15, h = l >> 4, g = n & 7, d = 2 * jp + (n >> 3);
  uint32_t wv[4] = {0, 0, 0, 0};
  if (d < P) {
    for (int t = 0; t < 16; t++) {
      const int slot = slot_tab[((size_t)T * 64 + 16 * h + t) * 8 + g];
      if (slot < 0) continue;
      const u64 v = pt[((size_t)slot * pqn + r) * N + x];
      const u64 bal = P == 5 ? Balanced<5>::of(v, pi.q) : Balanced<8>::of(v, pi.q);
      const uint32_t byte = (uint32_t)(bal >> (8 * d)) & 0xFFu;
      wv[t >> 2] |= byte << (8 * (t & 3));
    }
  }
  uint32_t *o = (uint32_t *)(ptm + (trx * 4 + jp) * 1024 + l * 16);
  o[0] = wv[0];
  o[1] = wv[1];
  o[2] = wv[2];
  o[3] = wv[3];
}

// Plain a_j of a seeded key (REDC of the Montgomery-form value) on every prime.
__global__ __launch_bounds__(TPB) void key_uniform_kernel(u64 seed, int j, u64 *out, const PrimeInfo *pinfo,
                                                          int N) {
  const int x = blockIdx.x * TPB + threadIdx.x, p = blockIdx.y;
  const PrimeInfo pi = pinfo[p];
  out[(size_t)p * N + x] = redc(key_uniform_mont(seed, j, p, x, pi), 0, pi.q, pi.qn);
}

dim3 ew_grid(const helrm_ctx *ctx, int rows) { return dim3(ctx->N / TPB, rows); }

}  // namespace

// ---------------------------------------------------------------- launchers

int launch_poly_op(helrm_ctx *ctx, int op, const u64 *a, const u64 *b, u64 *out, const LimbList &ll,
                   int batch, hipStream_t s) {
  if (ll.n * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(poly_op_kernel, ew_grid(ctx, ll.n * batch), dim3(TPB), 0, s, op, a, b, out, ll,
                     ctx->d_pinfo, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_mul_scalar(helrm_ctx *ctx, const u64 *a, const u64 *scal, u64 *out, const LimbList &ll,
                      int batch, hipStream_t s) {
  if (ll.n > 64) {
    set_error("mul_scalar: at most 64 limbs per launch");
    return HELRM_EINVAL;
  }
  ScalarArgs sc;
  for (int i = 0; i < ll.n; i++) {
    const u64 q = ctx->primes[ll.prime[i]];
    const u64 w = scal[i] % q;
    sc.c[i].w = w;
    sc.c[i].wp = (u64)(((u128)w << 64) / q);
  }
  if (ll.n * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(mul_scalar_kernel, ew_grid(ctx, ll.n * batch), dim3(TPB), 0, s, a, out, ll, sc,
                     ctx->d_pinfo, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_from_signed(helrm_ctx *ctx, const int64_t *in, u64 *out, const LimbList &ll, int batch,
                       hipStream_t s) {
  if (ll.n * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(from_signed_kernel, ew_grid(ctx, ll.n * batch), dim3(TPB), 0, s, in, out, ll,
                     ctx->d_pinfo, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

__global__ __launch_bounds__(TPB) void pack_key_kernel(const u64 *key, uint32_t *lo, uint8_t *hi, int keyl, int N) {
  const int x = blockIdx.x * TPB + threadIdx.x;
  const int j = blockIdx.y / keyl, p = blockIdx.y % keyl;
  const u64 v = key[((size_t)(2 * j) * keyl + p) * N + x];
  const size_t i = ((size_t)j * keyl + p) * N + x;
  lo[i] = (uint32_t)v;
  hi[i] = (uint8_t)(v >> 32);
}

int launch_pack_key(helrm_ctx *ctx, u64 *key, hipStream_t s) {
  const int keyl = ctx->L + 1 + ctx->K;
  uint32_t *lo = (uint32_t *)(key + key_words(ctx->dnum, keyl, ctx->N));
  uint8_t *hi = (uint8_t *)(lo + (size_t)ctx->dnum * keyl * ctx->N);
  hipLaunchKernelGGL(pack_key_kernel, ew_grid(ctx, ctx->dnum * keyl), dim3(TPB), 0, s, key, lo, hi, keyl, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

__global__ __launch_bounds__(TPB) void pack40_kernel(const u64 *in, uint32_t *lo, uint8_t *hi, size_t n) {
  const size_t i = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const u64 v = in[i];
  lo[i] = (uint32_t)v;
  hi[i] = (uint8_t)(v >> 32);
}

int launch_pack_pt(u64 *pt, size_t words, hipStream_t s) {
  if (words == 0) return HELRM_OK;
  uint32_t *lo = (uint32_t *)(pt + words);
  uint8_t *hi = (uint8_t *)(lo + words);
  hipLaunchKernelGGL(pack40_kernel, dim3((unsigned)((words + TPB - 1) / TPB)), dim3(TPB), 0, s, pt, lo, hi, words);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_to_mont(helrm_ctx *ctx, u64 *data, const LimbList &ll, int batch, hipStream_t s) {
  if (ll.n * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(to_mont_kernel, ew_grid(ctx, ll.n * batch), dim3(TPB), 0, s, data, ll, ctx->d_pinfo,
                     ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_copy_limbs(const u64 *src, u64 *dst, const LimbList &ll, int batch, int N, hipStream_t s) {
  if (ll.n * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(copy_limbs_kernel, dim3(N / TPB, ll.n * batch), dim3(TPB), 0, s, src, dst, ll, N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_automorph(helrm_ctx *ctx, const u64 *in, u64 *out, uint32_t galois, int n_limbs, int batch,
                     hipStream_t s) {
  if (n_limbs * batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(automorph_kernel, ew_grid(ctx, n_limbs * batch), dim3(TPB), 0, s, in, out,
                     (unsigned)galois, ctx->logn);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_conv(helrm_ctx *ctx, const ConvSpec *specs, int nspecs, const u64 *src, int src_bstride,
                const u64 *copy_src, int copy_bstride, u64 *dst, int dst_bstride, int batch, hipStream_t s) {
  if (nspecs > HELRM_MAX_CONV_JOBS) {
    set_error("conv: at most %d jobs per launch", HELRM_MAX_CONV_JOBS);
    return HELRM_EINVAL;
  }
  if (batch == 0 || nspecs == 0) return HELRM_OK;
  // jobs of one launch share the input count; split by it, except that a list
  // with a fused ModDown runs as one launch of the largest count
  bool any_pre = false;
  for (int k = 0; k < nspecs; k++) any_pre = any_pre || specs[k].pre;
  int done = 0;
  while (done < nspecs) {
    int nin = specs[done].t->nin;
    int end = done;
    if (any_pre) {
      for (end = done; end < nspecs; end++) nin = std::max(nin, specs[end].t->nin);
    } else {
      while (end < nspecs && specs[end].t->nin == nin) end++;
    }
    ConvJobs J;
    memset(&J, 0, sizeof J);
    J.njobs = end - done;
    J.nchunks = 1;
    double words = 0, macs = 0;
    for (int k = done; k < end; k++) {
      const ConvSpec &sp = specs[k];
      ConvJob &jb = J.j[k - done];
      jb.t = *sp.t;
      jb.src_off0 = sp.src_off0;
      for (int r = 0; r < sp.t->nout; r++) jb.dst_off[r] = sp.dst_off[r];
      jb.ncopy = sp.ncopy;
      for (int c = 0; c < sp.ncopy; c++) {
        jb.copy_src_off[c] = sp.copy_src_off[c];
        jb.copy_dst_off[c] = sp.copy_dst_off[c];
      }
      jb.fin = sp.fin;
      jb.fin_off0 = sp.fin_off0;
      jb.qlinv = sp.qlinv;
      jb.pre = sp.pre ? 1 : 0;
      if (sp.pre) {
        if (sp.pre->nin != nin || sp.pre_col0 + sp.t->nin > sp.pre->nout) {
          set_error("conv: a fused ModDown needs as many special primes as inputs");
          return HELRM_EINVAL;
        }
        jb.pre_src0 = sp.pre_src0;
        jb.pre_a0 = sp.pre_a0;
        jb.pre_col0 = sp.pre_col0;
        jb.pre_dst0 = sp.pre_dst0;
        jb.pre_ncol = sp.pre->nout;
        jb.pre_prime0 = sp.pre->in_prime[0];
        for (int k = 1; k < nin; k++)
          if (sp.pre->in_prime[k] != jb.pre_prime0 + k) {
            set_error("conv: a fused ModDown needs consecutive special primes");
            return HELRM_EINVAL;
          }
        jb.pre_hat_inv = sp.pre->hat_inv;
        jb.pre_hat_mont = sp.pre->hat_mont;
      }
      const int nw = sp.fin == CONV_FIN_RESCALE ? sp.t->nout - 1 : sp.t->nout;
      // with a ModDown in front: K special and nin A limbs read, nin z limbs written
      words += (sp.pre ? 3.0 * sp.t->nin : sp.t->nin) + nw + 2.0 * sp.ncopy +
               (sp.fin != CONV_FIN_NONE ? sp.t->nout : 0);
      macs += (double)sp.t->nin * (sp.t->nout + (sp.pre ? sp.t->nin : 0));
    }
    // output chunks: enough workgroups for several waves per SIMD, at least
    // four outputs per chunk
    int minout = HELRM_MAX_PRIMES;
    for (int k = 0; k < J.njobs; k++)
      minout = std::min(minout, J.j[k].t.nout - (J.j[k].fin == CONV_FIN_RESCALE ? 1 : 0));
    const long base = (long)(ctx->N / CONV_TPB) * batch * J.njobs;
    bool pre = false;
    for (int k = 0; k < J.njobs; k++) pre = pre || J.j[k].pre;
    if (!pre && ctx->tune_conv_wgs > 0 && base < ctx->tune_conv_wgs)
      J.nchunks = (int)std::max(1L, std::min((long)std::max(1, minout / 4),
                                             (ctx->tune_conv_wgs + base - 1) / base));
    dim3 grid(ctx->N / CONV_TPB * J.nchunks, 1, batch * J.njobs);
    KTimer tm(ctx, s);
#define CONV(NIN_)                                                                                     \
  if (pre)                                                                                             \
    hipLaunchKernelGGL((conv_kernel<NIN_, true>), grid, dim3(CONV_TPB), 0, s, J, src, src_bstride,      \
                       copy_src, copy_bstride, dst, dst_bstride, ctx->d_pinfo, ctx->N);                \
  else                                                                                                 \
    hipLaunchKernelGGL((conv_kernel<NIN_, false>), grid, dim3(CONV_TPB), 0, s, J, src, src_bstride,     \
                       copy_src, copy_bstride, dst, dst_bstride, ctx->d_pinfo, ctx->N)
    switch (nin) {
      case 1: CONV(1); break;
      case 2: CONV(2); break;
      case 3: CONV(3); break;
      case 4: CONV(4); break;
      case 5: CONV(5); break;
      case 6: CONV(6); break;
      case 7: CONV(7); break;
      case 8: CONV(8); break;
      case 9: CONV(9); break;
      case 10: CONV(10); break;
      case 11: CONV(11); break;
      case 12: CONV(12); break;
      case 13: CONV(13); break;
      case 14: CONV(14); break;
      case 15: CONV(15); break;
      case 16: CONV(16); break;
      default:
        set_error("conv: %d inputs unsupported", nin);
        return HELRM_EINVAL;
    }
#undef CONV
    tm.lap(TK_CONV, words * 8.0 * ctx->N * batch, macs * ctx->N * batch);
    HIP_TRY(hipGetLastError());
    done = end;
  }
  return HELRM_OK;
}

int launch_sub_mul(helrm_ctx *ctx, const u64 *a, const u64 *b, int b_bstride, u64 *out,
                   const LimbList &ll, const TW *consts, int batch, hipStream_t s) {
  if (ll.n * batch == 0) return HELRM_OK;
  KTimer tm(ctx, s);
  hipLaunchKernelGGL(sub_mul_kernel, ew_grid(ctx, ll.n * batch), dim3(TPB), 0, s, a, b, out, ll, consts,
                     ctx->d_pinfo, ctx->N, b_bstride);
  tm.lap(TK_SUB_MUL, 24.0 * ctx->N * ll.n * batch, (double)ctx->N * ll.n * batch);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_rescale_spread(helrm_ctx *ctx, const u64 *top, u64 *out, int level, int batch, hipStream_t s) {
  if (batch == 0 || level == 0) return HELRM_OK;
  hipLaunchKernelGGL(rescale_spread_kernel, ew_grid(ctx, 2 * batch * level), dim3(TPB), 0, s, top, out,
                     level, ctx->d_pinfo, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int pick_bt(int batch, int cap) {
  int bt = 1;
  while (bt < cap && bt < batch) bt *= 2;
  return bt;
}

// Key words per coefficient of one rotation read from memory, summed over
// the PQ limbs of `level`: 2 beta (both halves), less beta where the kernel
// regenerates the a_j halves (primes below 2^40, or every prime with
// gen_wide), the b halves counted at 5/8 where read from their 40-bit planes.
double key_limb_words(const helrm_ctx *ctx, int level, bool gen, int gen_wide, double beta, bool packed) {
  // b halves: 5 bytes per word on primes below 2^40 where the kernel reads
  // their 40-bit planes (packed)
  double w = 0;
  for (int r = 0; r < level + 1 + ctx->K; r++) {
    const bool small = ctx->primes[ctx->pq_prime(r, level)] < SPLIT_MAC_LIMIT;
    w += (small && packed ? beta * 5.0 / 8.0 : beta) + (gen && (small || gen_wide) ? 0.0 : beta);
  }
  return w;
}

int launch_ks_accumulate(helrm_ctx *ctx, int level, const KsTerm *terms, int n_terms,
                         size_t digits_bstride, size_t c0_bstride, const u64 *base, size_t base_bstride,
                         u64 *out, size_t out_bstride, int batch, hipStream_t s) {
  LevelGeom G{level, ctx->n_digits(level), level + 1 + ctx->K, ctx->L + 1 + ctx->K, ctx->logn, ctx->dnum, ctx->tune_limb_xcd,
               ctx->tune_gen_key_a == 2 ? 1 : 0, ctx->tune_ks_chain ? ctx->d_chain256 : nullptr};
  if (G.beta > MAXBETA || G.beta < 1) {
    set_error("key switching with %d digits (1 to %d supported)", G.beta, MAXBETA);
    return HELRM_EINVAL;
  }
  if (batch == 0) return HELRM_OK;
  const int bt = pick_bt(batch, ctx->tune_ks_tile);
  const int ntiles = (batch + bt - 1) / bt;
  const int grid = (ctx->N / TPB) * G.pqn * ntiles;
  // long term lists run as several launches: the first writes `out` (with the
  // lifted base), the others add to it
  for (int t0 = 0; t0 == 0 || t0 < n_terms; t0 += HELRM_MAX_TERMS) {
    const int nt_i = std::min(HELRM_MAX_TERMS, n_terms - t0);
    KsArgs T;
    T.n = nt_i;
    T.accum = t0 > 0;
    bool seeded = true;
    for (int i = 0; i < nt_i; i++) {
      T.digits[i] = terms[t0 + i].digits;
      T.c0[i] = terms[t0 + i].c0;
      T.key[i] = terms[t0 + i].key;
      T.gal[i] = terms[t0 + i].galois;
      T.seed[i] = terms[t0 + i].seed;
      seeded = seeded && terms[t0 + i].seeded;
    }
    // one ciphertext per thread: every key word is used once, so regenerating
    // the a_j halves halves the key traffic (on primes below 2^40, where the
    // generator is cheap, unless gen_key_a = 2)
    const bool gen = bt == 1 && seeded && nt_i > 0 && ctx->tune_gen_key_a >= 1;
    const u64 *bse = t0 == 0 ? base : nullptr;
    // per coefficient of a Q limb: terms * 3 beta words (digit, key b, key a) + the c0 words
    // + 2 base words + 2 output words (4 when adding to out); special limbs: no c0 / base
    // words.  Keys count once per launch, the rest once per ciphertext.
    double nc0 = 0;
    for (int i = 0; i < nt_i; i++) nc0 += T.c0[i] ? 1 : 0;
    const double qn = level + 1, K = ctx->K, nt = nt_i, beta = G.beta, B = batch, ow = T.accum ? 4 : 2;
    // key words per term and coefficient read from memory, summed over the limbs
    const double kl = key_limb_words(ctx, level, gen, G.gen_wide, beta, true);
    const double words = nt * kl + qn * B * (nt * beta + nc0 + (bse ? 2 : 0) + ow) + K * B * (nt * beta + ow);
    KTimer tm(ctx, s);
#define KSACC(BT_, BETA_, GEN_)                                                                        \
  hipLaunchKernelGGL((ks_acc_kernel<BT_, BETA_, GEN_>), dim3(grid), dim3(TPB), 0, s, T, G, ctx->L,      \
                     batch, ntiles, digits_bstride, c0_bstride, bse, base_bstride, out, out_bstride,    \
                     ctx->d_pinfo)
#define KSACC_B(BT_, GEN_)                      \
  switch (G.beta) {                             \
    case 1: KSACC(BT_, 1, GEN_); break;         \
    case 2: KSACC(BT_, 2, GEN_); break;         \
    case 3: KSACC(BT_, 3, GEN_); break;         \
    default: KSACC(BT_, 4, GEN_); break;        \
  }
    if (gen) {
      KSACC_B(1, true);
    } else {
      switch (bt) {
        case 1: KSACC_B(1, false); break;
        case 2: KSACC_B(2, false); break;
        default: KSACC_B(4, false); break;
      }
    }
#undef KSACC_B
#undef KSACC
    tm.lap(TK_KS_ACC, 8.0 * ctx->N * words, 2.0 * nt * beta * ctx->N * B * (qn + K));
    HIP_TRY(hipGetLastError());
  }
  return HELRM_OK;
}

int launch_ptm_pack(helrm_ctx *ctx, const helrm_plan *plan, const int *slot_tab, hipStream_t s) {
  const int pqn = plan->level + 1 + ctx->K;
  const size_t threads = (size_t)pqn * ctx->N * 256;
  hipLaunchKernelGGL(ptm_pack_kernel, dim3((unsigned)(threads / 256), plan->ptm_tiles), dim3(256), 0, s, plan->d_pt,
                     slot_tab,
                     plan->d_ptm, pqn, plan->level, ctx->L, ctx->N, ctx->d_pinfo);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_wfold_pack(helrm_ctx *ctx, helrm_plan *plan, int T, hipStream_t s) {
  const int pqn = plan->level + 1 + ctx->K, n1 = plan->n1;
  FoldPack FP;
  memset(&FP, 0, sizeof FP);
  FP.kc = plan->wm_kc;
  FP.beta = ctx->n_digits(plan->level);
  FP.ng = std::min(HELRM_MAX_GTILE, plan->n2 - T * HELRM_MAX_GTILE);
  for (int r = 0; r < pqn; r++) {
    FP.off[r] = (unsigned)plan->wm_off[r];
    FP.planes[r] = (unsigned char)plan->wm_planes[r];
  }
  // the tile's baby steps, in the baby-step launch's order (b = 0 first)
  int ns = 0;
  for (int b : plan->babies) {
    bool any = false;
    for (int g = 0; g < FP.ng; g++)
      if (plan->slot[(size_t)(T * HELRM_MAX_GTILE + g) * n1 + b] >= 0) any = true;
    if (!any) continue;
    if (ns > HELRM_MAX_BABY) {
      set_error("key folding: too many baby steps in a giant tile");
      return HELRM_EINVAL;
    }
    for (int g = 0; g < 8; g++)
      FP.slot[ns][g] = g < FP.ng ? (short)plan->slot[(size_t)(T * HELRM_MAX_GTILE + g) * n1 + b] : (short)-1;
    if (b == 0 && ns == 0) {
      FP.has0 = 1;
    } else {
      const uint32_t gal = galois_of_step(ctx, (long)plan->sign * b);
      auto it = ctx->keys.find(gal);
      if (it == ctx->keys.end()) {
        set_error("key folding: no evaluation key for rotation %d", b);
        return HELRM_EINVAL;
      }
      FP.key[ns - FP.has0] = it->second.d;
    }
    ns++;
  }
  FP.nslot = ns;
  const size_t threads = (size_t)pqn * ctx->N * 8 * 64;
  hipLaunchKernelGGL(wfold_pack_kernel, dim3((unsigned)(threads / 256), FP.kc), dim3(256), 0, s, FP, plan->d_pt,
                     plan->d_wm + (size_t)T * plan->wm_tile_bytes, pqn, plan->level, ctx->L, ctx->logn,
                     ctx->L + 1 + ctx->K, ctx->d_pinfo);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_baby_mac(helrm_ctx *ctx, const helrm_plan *plan, const u64 *digits, size_t digits_bstride,
                    const u64 *ct, size_t ct_bstride, u64 *X, size_t x_bstride, int g0, int ng, int batch,
                    hipStream_t s, bool accum, bool force, uint32_t *fold_ws) {
  if (ng > HELRM_MAX_GTILE) {
    set_error("baby_mac: at most %d giant outputs per launch", HELRM_MAX_GTILE);
    return HELRM_EINVAL;
  }
  BabyArgs BA;
  BA.nrot = 0;
  BA.has0 = 0;
  bool seeded = true;
  for (int gi = 0; gi < HELRM_MAX_GTILE; gi++) BA.slot0[gi] = -1;
  double npt = 0;
  for (int b : plan->babies) {
    short sl[HELRM_MAX_GTILE];
    bool any = false;
    for (int gi = 0; gi < HELRM_MAX_GTILE; gi++) {
      sl[gi] = gi < ng ? (short)plan->slot[(size_t)(g0 + gi) * plan->n1 + b] : (short)-1;
      if (sl[gi] >= 0) {
        any = true;
        npt++;
      }
    }
    if (!any) continue;
    if (b == 0) {
      BA.has0 = 1;
      for (int gi = 0; gi < HELRM_MAX_GTILE; gi++) BA.slot0[gi] = sl[gi];
      continue;
    }
    if (BA.nrot >= HELRM_MAX_BABY) {
      set_error("baby_mac: at most %d baby steps", HELRM_MAX_BABY);
      return HELRM_EINVAL;
    }
    const uint32_t g = galois_of_step(ctx, (long)plan->sign * b);
    auto it = ctx->keys.find(g);
    if (it == ctx->keys.end()) {
      set_error("no evaluation key loaded for rotation %d (galois %llu)", b, (unsigned long long)g);
      return HELRM_EINVAL;
    }
    const int i = BA.nrot++;
    BA.key[i] = it->second.d;
    BA.gal[i] = (unsigned)g;
    BA.seed[i] = it->second.seed;
    seeded = seeded && it->second.seeded;
    for (int gi = 0; gi < HELRM_MAX_GTILE; gi++) BA.slot[i][gi] = sl[gi];
  }
  const int level = plan->level;
  LevelGeom G{level, ctx->n_digits(level), level + 1 + ctx->K, ctx->L + 1 + ctx->K, ctx->logn, ctx->dnum, ctx->tune_limb_xcd,
               ctx->tune_gen_key_a == 2 ? 1 : 0, ctx->tune_ks_chain ? ctx->d_chain256 : nullptr};
  if (G.beta > MAXBETA || G.beta < 1) {
    set_error("key switching with %d digits (1 to %d supported)", G.beta, MAXBETA);
    return HELRM_EINVAL;
  }
  if (batch == 0 || ng == 0 || (BA.nrot == 0 && !BA.has0 && !force)) return HELRM_OK;
  // algorithmic words per coefficient: keys and plaintexts once per launch, the rest per ciphertext
  const double nrot = BA.nrot, has0 = BA.has0;
  const double qn = level + 1, K = ctx->K, beta = G.beta, B = batch;
  const int gt = ng <= 1 ? 1 : ng <= 2 ? 2 : ng <= 4 ? 4 : 8;
  const double xw = accum ? 4 : 2;   // output words per giant (read as well when accumulating)
  // one ciphertext per thread and few giant outputs: the kernel streams keys,
  // so it regenerates their a_j halves instead of reading them
  const bool shared_path = ng >= 2 && batch >= 2 && ctx->tune_baby_share >= 2;
  const int bt_path = shared_path ? 0 : pick_bt(batch, gt >= 4 ? 1 : gt == 2 ? std::min(2, ctx->tune_baby_tile)
                                                                             : ctx->tune_baby_tile);
  const bool gen = !shared_path && bt_path == 1 && gt <= 2 && seeded && BA.nrot > 0 && ctx->tune_gen_key_a >= 1;
  const double kl = key_limb_words(ctx, level, gen, G.gen_wide, beta, !shared_path);
  // plaintext words per coefficient: 5 bytes on the 40-bit limbs of the per-thread kernel
  double pl = 0;
  for (int r = 0; r < level + 1 + ctx->K; r++)
    pl += !shared_path && ctx->primes[ctx->pq_prime(r, level)] < SPLIT_MAC_LIMIT ? 5.0 / 8.0 : 1.0;
  const double words = nrot * kl + pl * npt + qn * B * (nrot * (beta + 1) + 2 * has0 + xw * ng) +
                       K * B * (nrot * beta + xw * ng);
  KTimer tm(ctx, s);
  const bool fold = fold_ws && plan->d_wm && plan->wm_keys_gen == ctx->keys_gen && ctx->tune_baby_fold > 0 &&
                    batch >= ctx->tune_baby_fold && g0 % HELRM_MAX_GTILE == 0 &&
                    g0 / HELRM_MAX_GTILE < plan->wm_tiles && G.beta <= 3 && BA.nrot + BA.has0 <= 64;
  // the matrix-core MAC reads its plaintext operands padded to 64 baby steps
  // and 8 giant outputs: plans with few baby steps stay on the VALU kernels
  const bool mfma = !fold && plan->d_ptm && ctx->tune_baby_mfma > 0 && batch >= ctx->tune_baby_mfma &&
                    g0 % HELRM_MAX_GTILE == 0 && g0 / HELRM_MAX_GTILE < plan->ptm_tiles &&
                    BA.nrot + BA.has0 <= 64 && BA.nrot + BA.has0 >= ctx->tune_mfma_min_slots;
  if (fold) {
    // key-folded product on the matrix cores: the entries of every ciphertext
    // once, then one launch per digit count
    FoldRun FR;
    FR.nslot = BA.nrot + BA.has0;
    FR.has0 = BA.has0;
    FR.kc = plan->wm_kc;
    for (int i = 0; i < BA.nrot; i++) FR.gal[i] = BA.gal[i];
    for (int r = 0; r < G.pqn; r++) FR.off[r] = (unsigned)plan->wm_off[r];
    const uint8_t *wm = plan->d_wm + (size_t)(g0 / HELRM_MAX_GTILE) * plan->wm_tile_bytes;
    const size_t e_half = fold_entry_words(ctx, level) / 2, e_bs = 2 * e_half;
    {
      const size_t threads = (size_t)G.pqn * ctx->N;
#define FENT(BETA_)                                                                                         \
  hipLaunchKernelGGL((fold_entries_kernel<BETA_>), dim3((unsigned)((threads + 255) / 256), batch), dim3(256), 0, \
                     s, digits, digits_bstride, ct, ct_bstride, fold_ws, e_bs, e_half, FR, G, ctx->L, ctx->d_pinfo)
      switch (G.beta) {
        case 1: FENT(1); break;
        case 2: FENT(2); break;
        default: FENT(3); break;
      }
#undef FENT
    }
    for (int wide = 0; wide < 2; wide++) {
      LimbSel ls;
      ls.n = 0;
      for (int r = 0; r < G.pqn; r++)
        if ((ctx->primes[ctx->pq_prime(r, level)] >= SPLIT_MAC_LIMIT) == (wide == 1)) ls.r[ls.n++] = (unsigned char)r;
      if (ls.n == 0) continue;
      const int grid = (ctx->N / MF_XB) * ls.n;
      const u64 *chain = ctx->tune_block_chain ? ctx->d_block_chain : nullptr;
      // row tiles per group (knob), 1 when the batch has a single tile
      const bool two = batch > 16 && ((ctx->tune_fold_mp >> wide) & 1);
#define FOLDK(P_, MP_)                                                                                       \
  hipLaunchKernelGGL((baby_fold_kernel<P_, MP_>), dim3(grid), dim3(MF_TPB), 0, s, FR, G, ctx->L, batch, ls,  \
                     fold_ws, e_bs, e_half, wm, ng, X, x_bstride, accum ? 1 : 0, ctx->d_pinfo, chain)
      if (wide) {
        if (two) FOLDK(8, 2); else FOLDK(8, 1);
      } else {
        if (two) FOLDK(5, 2); else FOLDK(5, 1);
      }
#undef FOLDK
    }
  } else if (mfma) {
    // batched plaintext MAC on the matrix cores: one launch per digit count
    const int ntiles = (batch + MF_CT - 1) / MF_CT;
    const uint8_t *ptm = plan->d_ptm + (size_t)(g0 / HELRM_MAX_GTILE) * G.pqn * ctx->N * 4096;
    for (int wide = 0; wide < 2; wide++) {
      LimbSel ls;
      ls.n = 0;
      for (int r = 0; r < G.pqn; r++)
        if ((ctx->primes[ctx->pq_prime(r, level)] >= SPLIT_MAC_LIMIT) == (wide == 1)) ls.r[ls.n++] = (unsigned char)r;
      if (ls.n == 0) continue;
      const int grid = (ctx->N / MF_XB) * ls.n * ntiles;
#define BABYM(BETA_, P_)                                                                                 \
  hipLaunchKernelGGL((baby_mfma_kernel<BETA_, P_>), dim3(grid), dim3(MF_TPB), 0, s, BA, G, ctx->L, batch,  \
                     ntiles, ls, digits, digits_bstride, ct, ct_bstride, ptm, ng, X, x_bstride, accum ? 1 : 0, \
                     ctx->d_pinfo, nullptr)
#define BABYM_P(BETA_) \
  if (wide) BABYM(BETA_, 8); else BABYM(BETA_, 5);
      switch (G.beta) {
        case 1: BABYM_P(1); break;
        case 2: BABYM_P(2); break;
        case 3: BABYM_P(3); break;
        default: BABYM_P(4); break;
      }
#undef BABYM_P
#undef BABYM
    }
  } else if (ng >= 2 && batch >= 2 && ctx->tune_baby_share >= 2) {
    // several giant outputs and a batch: W ciphertexts per workgroup (blocks of 64 coefficients)
    G.chain = ctx->tune_ks_chain ? ctx->d_chain64 : nullptr;
    const int W = pick_bt(batch, ctx->tune_baby_share);
    const int gpw = (ng + W - 1) / W;
    const int ntiles = (batch + W - 1) / W;
    const int grid = (ctx->N / 64) * G.pqn * ntiles;
#define BABYS(W_, GPW_, BETA_)                                                                           \
  hipLaunchKernelGGL((baby_mac_shared_kernel<W_, GPW_, BETA_>), dim3(grid), dim3(64 * W_), 0, s, BA, G,  \
                     ctx->L, batch, ntiles, digits, digits_bstride, ct, ct_bstride, plan->d_pt, ng, X,     \
                     x_bstride, accum ? 1 : 0, ctx->d_pinfo)
#define BABYS_B(W_, GPW_)                     \
  switch (G.beta) {                           \
    case 1: BABYS(W_, GPW_, 1); break;        \
    case 2: BABYS(W_, GPW_, 2); break;        \
    case 3: BABYS(W_, GPW_, 3); break;        \
    default: BABYS(W_, GPW_, 4); break;       \
  }
    if (W == 8) {
      BABYS_B(8, 1);
    } else if (W == 4) {
      if (gpw == 1) BABYS_B(4, 1) else BABYS_B(4, 2)
    } else {
      if (gpw == 1) BABYS_B(2, 1) else if (gpw == 2) BABYS_B(2, 2) else BABYS_B(2, 4)
    }
#undef BABYS_B
#undef BABYS
  } else {
    const int bt = pick_bt(batch, gt >= 4 ? 1 : gt == 2 ? std::min(2, ctx->tune_baby_tile) : ctx->tune_baby_tile);
    const int ntiles = (batch + bt - 1) / bt;
    const int grid = (ctx->N / TPB) * G.pqn * ntiles;
#define BABY(GT_, BT_, BETA_, GEN_)                                                                      \
  hipLaunchKernelGGL((baby_mac_kernel<GT_, BT_, BETA_, GEN_>), dim3(grid), dim3(TPB), 0, s, BA, G,        \
                     ctx->L, batch, ntiles, digits, digits_bstride, ct, ct_bstride, plan->d_pt,            \
                     plan->pt_words, ng, X, x_bstride, accum ? 1 : 0, ctx->d_pinfo)
#define BABY_B(GT_, BT_, GEN_)                      \
  switch (G.beta) {                                 \
    case 1: BABY(GT_, BT_, 1, GEN_); break;         \
    case 2: BABY(GT_, BT_, 2, GEN_); break;         \
    case 3: BABY(GT_, BT_, 3, GEN_); break;         \
    default: BABY(GT_, BT_, 4, GEN_); break;        \
  }
    if (gen) {
      if (gt == 1) BABY_B(1, 1, true) else BABY_B(2, 1, true)
    } else if (gt == 1) {
      if (bt == 1) BABY_B(1, 1, false) else if (bt == 2) BABY_B(1, 2, false) else BABY_B(1, 4, false)
    } else if (gt == 2) {
      if (bt == 1) BABY_B(2, 1, false) else BABY_B(2, 2, false)
    } else if (gt == 4) {
      BABY_B(4, 1, false);
    } else {
      BABY_B(8, 1, false);
    }
#undef BABY_B
#undef BABY
  }
  // bytes the matrix-core paths move: per ciphertext its digits (and c0) and
  // giant outputs; the key-folded product streams the folded words once and
  // the entries (written by the entries pass, read back once: the
  // per-rotation gathers hit the caches); the other reads every rotation's
  // key and the plaintext digits once per tile of 8 ciphertexts
  const double Nd = ctx->N, pqn = qn + K, per_ct = Nd * 8.0 * (qn * (beta + 1) + K * beta + xw * ng * pqn);
  const double ops = (2.0 * nrot * beta + 2.0 * npt) * Nd * B * pqn;
  if (fold) {
    tm.lap(TK_BABY_FOLD, (double)plan->wm_tile_bytes + B * (per_ct + 8.0 * fold_entry_words(ctx, level)), ops);
  } else if (mfma) {
    double njp = 0;
    for (int r = 0; r < G.pqn; r++) njp += ctx->primes[ctx->pq_prime(r, level)] >= SPLIT_MAC_LIMIT ? 4 : 3;
    const double tiles = (batch + MF_CT - 1) / MF_CT;
    tm.lap(TK_BABY_MFMA, tiles * Nd * (16.0 * nrot * beta * pqn + 1024.0 * njp) + B * per_ct, ops);
  } else {
    tm.lap(TK_BABY_MAC, 8.0 * ctx->N * words, ops);
  }
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_tensor(helrm_ctx *ctx, const u64 *a, const u64 *b, u64 *d, int level, int batch, hipStream_t s) {
  const int qn = level + 1;
  if (batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(tensor_kernel, ew_grid(ctx, qn * batch), dim3(TPB), 0, s, a, b, d, qn, ctx->d_pinfo,
                     ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_add_plain(helrm_ctx *ctx, const u64 *ct, const u64 *pt, u64 *out, int level, int batch,
                     hipStream_t s) {
  const int qn = level + 1;
  if (batch == 0) return HELRM_OK;
  hipLaunchKernelGGL(add_plain_kernel, ew_grid(ctx, 2 * qn * batch), dim3(TPB), 0, s, ct, pt, out, qn,
                     ctx->d_pinfo, ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

int launch_key_uniform(helrm_ctx *ctx, u64 seed, int digit, u64 *out, hipStream_t s) {
  const int kl = ctx->L + 1 + ctx->K;
  hipLaunchKernelGGL(key_uniform_kernel, ew_grid(ctx, kl), dim3(TPB), 0, s, seed, digit, out, ctx->d_pinfo,
                     ctx->N);
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

// ---------------------------------------------------------------- ALU calibration
//
// Issue-rate ceilings of the two instructions the library's modular products
// are built from: the 32x32->64 integer multiply-add (v_mad_u64_u32: every
// Shoup, Montgomery and split product) and the fp64 FMA (the exact products
// of the small-prime NTT).  Each thread runs 16 independent chains with no
// memory access inside the loop; the result is written out so that nothing is
// optimised away.
__global__ __launch_bounds__(256) void calib_mad_kernel(const u64 *seed, u64 *out, int iters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  u64 a[16];
  uint32_t y[16];
#pragma unroll
  for (int k = 0; k < 16; k++) {
    a[k] = seed[(t + k) & 63];
    y[k] = (uint32_t)seed[64 + ((t + 5 * k) & 63)] | 1u;
  }
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int r = 0; r < 8; r++)
#pragma unroll
      for (int k = 0; k < 16; k++) a[k] = (u64)(uint32_t)a[k] * y[k] + a[k];
  }
  u64 acc = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) acc ^= a[k];
  out[t] = acc;
}

__global__ __launch_bounds__(256) void calib_fma_kernel(const u64 *seed, u64 *out, int iters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double d[16], c[16];
  const double m = 0.9990234375;   // d += c m: finite for any iteration count used here
#pragma unroll
  for (int k = 0; k < 16; k++) {
    d[k] = (double)(seed[(t + k) & 63] >> 40);
    c[k] = (double)(seed[64 + ((t + 5 * k) & 63)] >> 44);
  }
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int r = 0; r < 8; r++)
#pragma unroll
      for (int k = 0; k < 16; k++) d[k] = __fma_rn(c[k], m, d[k]);
  }
  u64 acc = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) acc ^= (u64)__double_as_longlong(d[k]);
  out[t] = acc;
}

int calibrate_instr(int kind, hipStream_t s, double *per_s) {
  const int blocks = 256 * 16, iters = 256;
  const size_t threads = (size_t)blocks * 256;
  u64 *buf = nullptr;
  HIP_TRY(hipMalloc(&buf, (128 + threads) * sizeof(u64)));
  std::vector<u64> seed(128);
  u64 z = 0x13198A2E03707344ull;
  for (auto &v : seed) {
    z = z * 6364136223846793005ull + 1442695040888963407ull;
    v = z;
  }
  int rc = HELRM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMemcpy(buf, seed.data(), 128 * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    set_error("calibration set-up failed");
    rc = HELRM_EHIP;
  } else {
    for (int rep = 0; rep < 2; rep++) {
      if (rep == 1) (void)hipEventRecord(e0, s);
      if (kind == 0)
        hipLaunchKernelGGL(calib_mad_kernel, dim3(blocks), dim3(256), 0, s, buf, buf + 128, iters);
      else
        hipLaunchKernelGGL(calib_fma_kernel, dim3(blocks), dim3(256), 0, s, buf, buf + 128, iters);
    }
    (void)hipEventRecord(e1, s);
    float ms = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0) {
      (void)hipGetLastError();
      set_error("calibration launch failed");
      rc = HELRM_EHIP;
    } else {
      *per_s = (double)threads * iters * 8 * 16 / (ms * 1e-3);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return rc;
}
