// Negacyclic NTT / inverse NTT over RNS limbs for gfx950.
//
// Forward transform: out[j] = a(psi^(2 brv(j)+1)) mod q, the evaluation form
// used throughout the library (Cooley-Tukey with the bit-reversed table of psi
// powers, decimation in time, output in bit-reversed order).  The inverse is
// the Gentleman-Sande transform with psi^-1 powers followed by N^-1.
//
// A limb of N = R*R points (R = E*E, E = 2^H) is transformed in two passes:
//   * "column" pass: the R sub-transforms {c + R r : r < R} (stride R),
//   * "block"  pass: the R contiguous blocks {R b + s : s < R}.
// Each workgroup owns W sub-transforms; each thread holds E residues
// in registers and runs H butterfly stages on them, the workgroup exchanges
// the residues through LDS (swizzled against bank conflicts) and the thread
// runs the other H stages.  Global loads and stores are coalesced: in the
// column pass consecutive lanes own consecutive columns, in the block pass
// consecutive lanes own consecutive elements.  Primes of 41 bits and more
// take Harvey's lazy integer butterflies with Shoup twiddle products; smaller
// primes take signed fp64 butterflies with exact products and no reductions
// inside a pass (the policies below state the bounds).  Only the last pass
// reduces to [0,q); between the passes the lazy values go through HBM.
#include "common.h"

namespace {

// Shoup product with a three-term quotient: for y = y1 2^32 + y0 and
// w' = p1 2^32 + p0, floor(y w' / 2^64) is y1 p1 + hi(y1 p0) + hi(y0 p1)
// plus 0, 1 or 2 (the dropped low terms are below 3 2^64), so
// y w - qh q lies in [0, 4q) for any 64-bit y (Shoup: [0, 2q) with the exact
// quotient).  NEG forms it as y w + qh (2^64 - q) mod 2^64 (nq = 2^64 - q):
// both products go through the 32-bit multiply-adds into one sum with no
// borrow chain; fewer instructions, more live registers.
template <bool NEG>
__device__ __forceinline__ u64 shoup_lazy4(u64 y, u64 w, u64 wp, u64 q, u64 nq) {
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32), p0 = (uint32_t)wp, p1 = (uint32_t)(wp >> 32);
  const u64 qh = (u64)y1 * p1 + __umulhi(y1, p0) + __umulhi(y0, p1);
  if (!NEG) return y * w - qh * q;
  const uint32_t h0 = (uint32_t)qh, h1 = (uint32_t)(qh >> 32);
  const uint32_t w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32), n0 = (uint32_t)nq, n1 = (uint32_t)(nq >> 32);
  const u64 lo = (u64)y0 * w0 + (u64)h0 * n0;
  const uint32_t hi = (uint32_t)(lo >> 32) + y0 * w1 + y1 * w0 + h0 * n1 + h1 * n0;
  return ((u64)hi << 32) | (uint32_t)lo;
}

// Workgroup shape of one pass.  The column pass keeps WC consecutive columns
// per workgroup (WC words per row contiguous in HBM); the block pass keeps WB
// blocks.  Small workgroups let a launch of a few limbs fill 256 CUs.
template <int H, bool COLS, int W_ = (COLS ? 16 : 8)>
struct Shape {
  static constexpr int E = 1 << H;                    // residues per thread
  static constexpr int R = E * E;                     // sub-transform length
  static constexpr int N = R * R;                     // ring degree
  static constexpr int W = W_;                        // sub-transforms per workgroup
  static constexpr int T = W * E;                     // threads per workgroup
  static constexpr int WPL = R / W;                   // workgroups per limb
  // column pass: row stride E*W + W keeps the lane groups of a wave on
  // distinct bank halves; block pass: stride R + 16 plus an XOR swizzle.
  static constexpr int LDS = COLS ? (R * W + E * W) : (W * (R + 16));
};

// LDS index of element s of sub-transform w (block pass): XOR-swizzle the
// high H bits into the low H bits so both access patterns spread over banks.
template <int H>
__device__ __forceinline__ int blk_idx(int w, int s) {
  constexpr int E = 1 << H, R = E * E;
  return w * (R + 16) + (s ^ ((s >> H) & (E - 1)));
}

// LDS index of element r of column w (column pass, W columns per workgroup).
template <int H, int W>
__device__ __forceinline__ int col_idx(int w, int r) {
  return r * W + w + (r >> H) * W;
}

// ---------------------------------------------------------------- arithmetic policies
//
// IntA: residues as uint64 with Shoup twiddle products (primes below 2^60):
// lazy butterflies in the manner of Harvey on values in [0, 8q), with a
// three-term Shoup quotient (two 32-bit multiplies fewer per butterfly).
//
// FltA: residues as signed fp64 for primes below 2^41 (FLT_LIMIT).  The
// product a*w mod q is formed exactly: h = fl(a w) and l = fma(a, w, -h) give
// a w = h + l; qq = floor(h / q) (through the rounded reciprocal) is within
// one of floor(a w / q) while |a w / q| < 2^49; then fma(-qq, q, h) is the
// exact integer a w - qq q - l (its magnitude is below 2^53) and adding l
// gives r = a w - qq q exactly, with r in (-q, 2q).  No butterfly reduces or
// compares: a forward (Cooley-Tukey) stage adds at most 2q to the largest
// magnitude (x +- r), so 16 stages from [0, q) stay below 33q < 2^47; an
// inverse (Gentleman-Sande) stage at most doubles it (x + y), so each pass
// of 8 stages stays below 2^8 q < 2^49 and the first inverse pass ends with
// one floor reduction to [0, q].  The last step maps to [0, q) with
// r = v - q floor(v / q) (the quotient is exact for |v| < 2^50: its error is
// below 2^-44 < 1/q, except at exact multiples, where r may come out as q)
// and one conditional subtraction.  The intermediate between the two passes
// is stored as raw fp64 bits; fp64 FMA runs at the full VALU rate on gfx950.

constexpr u64 FLT_LIMIT = 1ull << 41;
constexpr long NTT_ORDER_MAX_LIMBS = 128;   // column passes of launches of up to this many limbs reorder them

// Integer butterflies on lazy values in [0, 8q) (q < 2^60, so 16 q < 2^64).
// Forward: X = x mod 4q in [0, 4q), T in [0, 4q): X + T and X - T + 4q stay
// in [0, 8q).  Inverse: x + y reduced once by 8q, and (x - y + 8q) w.  With
// NEG a multiple of q is subtracted by adding its negation mod 2^64.
template <bool NEG>
struct IntA {
  using V = u64;
  using T = TW;
  u64 q, q4, nq, nq4;   // nq = 2^64 - q, nq4 = 2^64 - 4q
  const TW *tw;
  __device__ __forceinline__ V load(u64 x) const { return x; }
  __device__ __forceinline__ u64 bits(V v) const { return v; }
  __device__ __forceinline__ V unbits(u64 b) const { return b; }
  // value stored between the passes (lazy)
  __device__ __forceinline__ u64 mid(V v, bool) const { return v; }
  __device__ __forceinline__ void ct(V &x, V &y, const T &t) const {
    const u64 X = x >= q4 ? (NEG ? x + nq4 : x - q4) : x;
    const u64 T = shoup_lazy4<NEG>(y, t.w, t.wp, q, nq);
    x = X + T;
    y = X - T + q4;
  }
  __device__ __forceinline__ void gs(V &x, V &y, const T &t) const {
    const u64 q8 = 2 * q4;
    u64 S = x + y;
    S = S >= q8 ? (NEG ? S + 2 * nq4 : S - q8) : S;
    const u64 D = x - y + q8;
    x = S;
    y = shoup_lazy4<NEG>(D, t.w, t.wp, q, nq);
  }
  // [0, 8q) -> [0, q)
  __device__ __forceinline__ u64 canon(V v) const {
    v = v >= q4 ? v - q4 : v;
    const u64 q2 = q4 >> 1;
    v = v >= q2 ? v - q2 : v;
    return v >= q ? v - q : v;
  }
  __device__ __forceinline__ u64 scale(V v, const PrimeInfo &pi) const { return shoup(v, pi.ninv, pi.ninv_p, q); }
  // fused finish: (a - y) c mod q for the transform output y, a in [0, q)
  __device__ __forceinline__ u64 finish(V v, u64 a, const TW &c) const {
    return shoup(sub_mod(a, canon(v), q), c.w, c.wp, q);
  }
};

struct FltA {
  using V = double;
  using T = double;
  double q, qinv;
  const double *tw;
  // 0 <= x < 2^52: x in the mantissa of 2^52, minus 2^52
  __device__ __forceinline__ V load(u64 x) const {
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
  }
  __device__ __forceinline__ u64 bits(V v) const { return (u64)__double_as_longlong(v); }
  __device__ __forceinline__ V unbits(u64 b) const { return __longlong_as_double((long long)b); }
  // a w - qq q in (-q, 2q) for |a w / q| < 2^49
  __device__ __forceinline__ double mm(double a, double w) const {
#pragma clang fp contract(off)
    const double h = a * w;
    const double l = __fma_rn(a, w, -h);
    const double qq = floor(h * qinv);
    return __fma_rn(-qq, q, h) + l;
  }
  // |v| < 2^50 -> [0, q]
  __device__ __forceinline__ double reduce(double v) const {
#pragma clang fp contract(off)
    return __fma_rn(-floor(v * qinv), q, v);
  }
  __device__ __forceinline__ u64 mid(V v, bool fwd) const { return bits(fwd ? v : reduce(v)); }
  __device__ __forceinline__ void ct(V &x, V &y, T t) const {
#pragma clang fp contract(off)
    const double r = mm(y, t);
    const double X = x;
    x = X + r;
    y = X - r;
  }
  __device__ __forceinline__ void gs(V &x, V &y, T t) const {
#pragma clang fp contract(off)
    const double S = x + y;
    const double D = x - y;
    x = S;
    y = mm(D, t);
  }
  // [0, q) as an integer: r + 2^52 has r in its low mantissa bits
  __device__ __forceinline__ u64 canon(V v) const {
#pragma clang fp contract(off)
    double r = reduce(v);
    r = r >= q ? r - q : r;
    return (u64)__double_as_longlong(r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
  }
  __device__ __forceinline__ u64 scale(V v, const PrimeInfo &pi) const { return canon(mm(v, pi.ninv_d)); }
  // fused finish: (a - y) c mod q for the lazy transform output y (|a - y| < 34 q)
  __device__ __forceinline__ u64 finish(V v, u64 a, const TW &c) const {
#pragma clang fp contract(off)
    return canon(mm(load(a) - v, (double)c.w));
  }
};

// Twiddles of one register phase.  Stage h (pairs k, k+h) uses m = E/(2h)
// consecutive table entries; in the "A" layout (element u + E k of the
// sub-transform) they start at m f, in the "B" layout (element E u + k) at
// m (E f + u).  Entry j = k/(2h) is read when the stage runs.
template <class A>
struct TwSrc {
  const typename A::T *tw;
  int base;   // f ("A" layout) or E f + u ("B" layout)
  __device__ __forceinline__ typename A::T operator()(int m, int j) const { return tw[m * base + j]; }
};

// H forward (Cooley-Tukey) stages on the E registers, h = E/2 .. 1.
template <int H, class A, class TS>
__device__ __forceinline__ void fwd_phase(typename A::V (&x)[1 << H], const A &ar, const TS &t) {
  constexpr int E = 1 << H;
#pragma unroll
  for (int h = E / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.ct(x[k], x[k + h], t(E / (2 * h), k / (2 * h)));
  }
}

// H inverse (Gentleman-Sande) stages, h = 1 .. E/2.
template <int H, class A>
__device__ __forceinline__ void inv_phase(typename A::V (&x)[1 << H], const A &ar, const TwSrc<A> &t) {
  constexpr int E = 1 << H;
#pragma unroll
  for (int h = 1; h <= E / 2; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.gs(x[k], x[k + h], t(E / (2 * h), k / (2 * h)));
  }
}

// Global index (within the limb) of register k of this thread for the pass's
// input; the data words are loaded before the prime is known.
template <int H, bool FWD, bool COLS, int WS>
__device__ __forceinline__ int in_index(int part, int k) {
  using S = Shape<H, COLS, WS>;
  constexpr int E = S::E, R = S::R, W = S::W;
  const int tid = threadIdx.x;
  if (COLS) {
    const int w = tid % W, u = tid / W;
    const int c = part * W + w;
    return FWD ? c + R * (u + E * k) : c + R * (E * u + k);
  }
  const int u = tid % E, w = tid / E;
  return R * (part * W + w) + u + E * k;
}

// The body of one pass for one arithmetic policy; raw[] holds the thread's
// input words (canonical residues for a first pass, the lazy intermediate
// for a second pass).  ar1 runs the first register phase of the forward
// block pass (the same arithmetic in another form), ar everything else.
template <int H, bool FWD, bool COLS, int WS, class A, class A1>
__device__ __forceinline__ void pass_body(const A &ar, const A1 &ar1, u64 *lds, const u64 (&raw)[1 << H], u64 *out,
                                          int part, int bat, int li, const PrimeInfo &pi, const NttEpi &epi) {
  using S = Shape<H, COLS, WS>;
  constexpr int E = S::E, R = S::R, N = S::N, W = S::W;
  using V = typename A::V;
  const int tid = threadIdx.x;
  V x[E];
  if (COLS) {
    const int w = tid % W, u = tid / W;
    const int c = part * W + w;
    if (FWD) {
      // first forward pass: stages m = 1 .. R/2 on column c
      const TwSrc<A> t1{ar.tw, 1}, t2{ar.tw, E + u};
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.load(raw[k]);
      fwd_phase<H>(x, ar, t1);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[col_idx<H, W>(w, E * u + k)]);
      fwd_phase<H>(x, ar, t2);
      // lazy values go to memory (integers below 8q, or fp64 bits)
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (E * u + k)] = ar.mid(x[k], true);
    } else {
      // last inverse pass: stages m = R/2 .. 1 on column c, then N^-1
      const TwSrc<A> t1{ar.tw, E + u}, t2{ar.tw, 1};
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(raw[k]);
      inv_phase<H>(x, ar, t1);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[col_idx<H, W>(w, u + E * k)]);
      inv_phase<H>(x, ar, t2);
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (u + E * k)] = ar.scale(x[k], pi);
    }
  } else {
    const int u = tid % E, w = tid / E;
    const int b = part * W + w;
    const int f = R + b;
    u64 *ob = out + (size_t)R * b;
    if (FWD) {
      // second forward pass (reads the lazy intermediate)
      const TwSrc<A> t1{ar.tw, f}, t2{ar.tw, E * f + u};
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(raw[k]);
      fwd_phase<H>(x, ar1, t1);
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, E * u + k)]);
      fwd_phase<H>(x, ar, t2);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
      if (epi.a && li < epi.n_fin) {
        // fused finish: out = (a - NTT(x)) * c  (ModDown: c = P^-1, rescale: c = q_l^-1)
        const int bo = bat / epi.inner, bi = bat % epi.inner;
        const u64 *ea = epi.a + ((size_t)bo * epi.a_bs + (size_t)bi * epi.a_cs + epi.a_off[li]) * (size_t)N +
                        (size_t)R * b;
        u64 *eo = epi.out + ((size_t)bo * epi.out_bs + (size_t)bi * epi.out_cs + epi.out_off[li]) * (size_t)N +
                  (size_t)R * b;
        const TW c = epi.c[li];
#pragma unroll
        for (int k = 0; k < E; k++) eo[u + E * k] = ar.finish(ar.unbits(lds[blk_idx<H>(w, u + E * k)]), ea[u + E * k], c);
      } else if (epi.dup && epi.dup_off[li] >= 0) {
        u64 *db = epi.dup + ((size_t)bat * epi.dup_bs + epi.dup_off[li]) * (size_t)N + (size_t)R * b;
#pragma unroll
        for (int k = 0; k < E; k++) {
          const u64 v = ar.canon(ar.unbits(lds[blk_idx<H>(w, u + E * k)]));
          ob[u + E * k] = v;
          db[u + E * k] = v;
        }
      } else {
#pragma unroll
        for (int k = 0; k < E; k++) ob[u + E * k] = ar.canon(ar.unbits(lds[blk_idx<H>(w, u + E * k)]));
      }
    } else {
      // first inverse pass (reads canonical residues)
      const TwSrc<A> t1{ar.tw, E * f + u}, t2{ar.tw, f};
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.load(raw[k]);
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, E * u + k)]);
      inv_phase<H>(x, ar, t1);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, u + E * k)]);
      inv_phase<H>(x, ar, t2);
      // values go to memory (integers below 8q, or fp64 bits in [0, q])
#pragma unroll
      for (int k = 0; k < E; k++) ob[u + E * k] = ar.mid(x[k], false);
    }
  }
}

// One pass of the transform.  FWD: column pass first (src -> dst), block pass
// second (in place, final reduction).  INV: block pass first, column pass
// second (in place, times N^-1).  Primes below 2^41 take the fp64 path.
template <int H, bool FWD, bool COLS, int WS>
__global__ __launch_bounds__((Shape<H, COLS, WS>::T)) void ntt_pass_kernel(const u64 *src, u64 *dst, LimbList ll,
                                                                         const TW *__restrict__ twtab,
                                                                         const double *__restrict__ twdtab,
                                                                         const PrimeInfo *__restrict__ pinfo,
                                                                         const NttEpi epi) {
  using S = Shape<H, COLS, WS>;
  constexpr int E = S::E, N = S::N, WPL = S::WPL;
  __shared__ u64 lds[S::LDS];
  const int limb_lin = blockIdx.x / WPL;
  const int part = blockIdx.x % WPL;
  const int bat = limb_lin / ll.n;
  const int li = limb_lin - bat * ll.n;
  const u64 *in = src + ((size_t)bat * ll.src_bstride + ll.src_off[li]) * (size_t)N;
  u64 *out = dst + ((size_t)bat * ll.dst_bstride + ll.dst_off[li]) * (size_t)N;
  // the data loads go out first, the prime's constants and twiddles follow
  u64 raw[E];
#pragma unroll
  for (int k = 0; k < E; k++) raw[k] = in[in_index<H, FWD, COLS, WS>(part, k)];
  const int p = ll.prime[li];
  const PrimeInfo pi = pinfo[p];
  if (pi.q < FLT_LIMIT) {
    FltA ar{pi.qd, pi.qinv_d, twdtab + (size_t)p * N};
    pass_body<H, FWD, COLS, WS>(ar, ar, lds, raw, out, part, bat, li, pi, epi);
  } else {
    // the second phase of the forward block pass (the one with the fused
    // epilogues) keeps the borrow-chain form: the other holds more registers
    // there and loses a wave per SIMD
    IntA<!(FWD && !COLS)> ar{pi.q, 4 * pi.q, 0 - pi.q, 0 - 4 * pi.q, twtab + (size_t)p * N};
    IntA<true> ar1{pi.q, 4 * pi.q, 0 - pi.q, 0 - 4 * pi.q, twtab + (size_t)p * N};
    pass_body<H, FWD, COLS, WS>(ar, ar1, lds, raw, out, part, bat, li, pi, epi);
  }
}

// The same limbs with those of primes of 41 bits and more first.  Their
// workgroups take the integer butterflies, about 2.5 times the instructions of
// the fp64 ones; dispatched first they start early and the shorter fp64
// workgroups fill in behind them.  Each entry keeps its own offsets, so the
// order changes nothing in the result (a fused epilogue, which is indexed by
// position, is never given a reordered list).
LimbList int_first(const helrm_ctx *ctx, const LimbList &ll) {
  LimbList o = ll;
  int k = 0;
  for (int pass = 0; pass < 2; pass++)
    for (int i = 0; i < ll.n; i++)
      if ((ctx->primes[ll.prime[i]] >= FLT_LIMIT) == (pass == 0)) {
        o.src_off[k] = ll.src_off[i];
        o.dst_off[k] = ll.dst_off[i];
        o.prime[k] = ll.prime[i];
        k++;
      }
  return o;
}

// Column-pass and block-pass workgroup widths (sub-transforms per workgroup):
// wider groups make longer contiguous runs in the column pass, narrower ones
// more workgroups for launches of few limbs.
template <int H, int WC, int WB>
int launch_ntt_hw(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                  hipStream_t s, const NttEpi &epi) {
  using SC = Shape<H, true, WC>;
  using SB = Shape<H, false, WB>;
  LimbList second = ll;
  for (int i = 0; i < ll.n; i++) second.src_off[i] = ll.dst_off[i];
  second.src_bstride = ll.dst_bstride;
  const int gc = ll.n * batch * SC::WPL, gb = ll.n * batch * SB::WPL;
  if (gc == 0) return HELRM_OK;
  // integer limbs first where measured faster: the inverse block pass, and
  // the column passes of launches that fill the chip about once
  const bool few = (long)ll.n * batch <= NTT_ORDER_MAX_LIMBS;
  // per pass and limb: N words read and written, (N/2) log2(R) butterflies
  const double limbs = (double)ll.n * batch;
  const double bytes = limbs * 16.0 * SC::N, ops = limbs * (SC::N / 2) * (2 * H);
  KTimer tm(ctx, s);
  if (forward) {
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, true, WC>), dim3(gc), dim3(SC::T), 0, s, src, dst,
                       few ? int_first(ctx, ll) : ll, ctx->d_tw_fwd, ctx->d_twd_fwd, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_FWD_COL, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, false, WB>), dim3(gb), dim3(SB::T), 0, s, dst, dst,
                       second, ctx->d_tw_fwd, ctx->d_twd_fwd, ctx->d_pinfo, epi);
    tm.lap(TK_NTT_FWD_BLK, bytes + (double)epi.n_fin * batch * 8.0 * SC::N, ops);
  } else {
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, false, WB>), dim3(gb), dim3(SB::T), 0, s, src, dst,
                       int_first(ctx, ll), ctx->d_tw_inv, ctx->d_twd_inv, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_INV_BLK, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, true, WC>), dim3(gc), dim3(SC::T), 0, s, dst, dst,
                       few ? int_first(ctx, second) : second, ctx->d_tw_inv, ctx->d_twd_inv, ctx->d_pinfo,
                       NttEpi{});
    tm.lap(TK_NTT_INV_COL, bytes, ops);
  }
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
}

template <int H>
int launch_ntt_h(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                 hipStream_t s, const NttEpi &epi) {
  // widths: the autotuner's choice, or by launch size (launches of few limbs
  // take the narrow shapes so they spread over more compute units)
  int wc = ctx->tune_ntt_col_w, wb = ctx->tune_ntt_blk_w;
  if (wc == 0) wc = (long)ll.n * batch < ctx->ntt_small_limbs ? 8 : 16;
  if (wb == 0) wb = (long)ll.n * batch < ctx->ntt_small_limbs ? 4 : 8;
  if (wc == 8 && wb == 4) return launch_ntt_hw<H, 8, 4>(ctx, src, dst, ll, batch, forward, s, epi);
  if (wc == 8) return launch_ntt_hw<H, 8, 8>(ctx, src, dst, ll, batch, forward, s, epi);
  if (wb == 4) return launch_ntt_hw<H, 16, 4>(ctx, src, dst, ll, batch, forward, s, epi);
  return launch_ntt_hw<H, 16, 8>(ctx, src, dst, ll, batch, forward, s, epi);
}

// ---------------------------------------------------------------- ALU calibration
//
// The ALU ceiling of the butterfly arithmetic: every thread keeps 16 residues
// and 16 twiddles in registers and repeats forward radix-16 phases (4 stages,
// 32 butterflies each) with the policy the passes use, with no memory access
// inside the loop.  The fp64 policy's magnitudes grow by at most 2q a stage,
// so every 4 phases (16 stages, as in a forward transform) the registers are
// brought back to [0, q], which the transform's last pass also does.  The
// result is written out so that nothing is optimised away.
struct RegTw {
  template <class T>
  struct Src {
    const T (&t)[16];
    __device__ __forceinline__ T operator()(int m, int j) const { return t[(m + j) & 15]; }
  };
};

template <class A>
__global__ __launch_bounds__(256) void calib_bfly_kernel(A ar, const u64 *seed, u64 *out, int iters) {
  using V = typename A::V;
  using T = typename A::T;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  V x[16];
  T w[16];
#pragma unroll
  for (int k = 0; k < 16; k++) {
    x[k] = ar.load(seed[(t + k) & 63] % ar.q_int());
    w[k] = ar.tw_of(seed[64 + ((t + 3 * k) & 63)] % ar.q_int(), seed[128 + ((t + 3 * k) & 63)]);
  }
  const RegTw::Src<T> src{w};
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int ph = 0; ph < 4; ph++) fwd_phase<4>(x, ar, src);
    ar.renorm(x);
  }
  u64 acc = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) acc ^= ar.bits(x[k]);
  out[t] = acc;
}

// Integer policy with the calibration hooks (values stay in [0, 8q)).
template <bool NEG>
struct IntCal : IntA<NEG> {
  __device__ __forceinline__ u64 q_int() const { return this->q; }
  __device__ __forceinline__ TW tw_of(u64 w, u64 wp) const { return TW{w, wp}; }
  __device__ __forceinline__ void renorm(u64 (&)[16]) const {}
};

struct FltCal : FltA {
  u64 qi;
  __device__ __forceinline__ u64 q_int() const { return qi; }
  __device__ __forceinline__ double tw_of(u64 w, u64) const { return (double)w; }
  __device__ __forceinline__ void renorm(double (&x)[16]) const {
#pragma unroll
    for (int k = 0; k < 16; k++) x[k] = reduce(x[k]);
  }
};

}  // namespace

// Butterflies per second of the register-resident loop above on prime q
// (fp64 policy below 2^41, integer policy from 2^41): one launch of
// blocks x 256 threads after one warm-up launch, timed with HIP events on s.
int calibrate_butterflies(helrm_ctx *ctx, u64 q, hipStream_t s, double *per_s) {
  const int blocks = 256 * 16, iters = 64;
  const size_t threads = (size_t)blocks * 256;
  u64 *buf = nullptr;
  HIP_TRY(hipMalloc(&buf, (192 + threads) * sizeof(u64)));
  std::vector<u64> seed(192);
  u64 z = 0x243F6A8885A308D3ull;
  for (auto &v : seed) {
    z = z * 6364136223846793005ull + 1442695040888963407ull;
    v = z;
  }
  // twiddle words below q with their Shoup quotients
  for (int k = 0; k < 64; k++) {
    seed[64 + k] %= q;
    seed[128 + k] = (u64)(((unsigned __int128)seed[64 + k] << 64) / q);
  }
  int rc = HELRM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMemcpy(buf, seed.data(), 192 * sizeof(u64), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    set_error("calibration set-up failed");
    rc = HELRM_EHIP;
  } else {
    for (int rep = 0; rep < 2; rep++) {
      if (rep == 1) (void)hipEventRecord(e0, s);
      if (q < FLT_LIMIT) {
        FltCal ar;
        ar.q = (double)q;
        ar.qinv = 1.0 / (double)q;
        ar.tw = nullptr;
        ar.qi = q;
        hipLaunchKernelGGL(calib_bfly_kernel<FltCal>, dim3(blocks), dim3(256), 0, s, ar, buf, buf + 192, iters);
      } else {
        IntCal<true> ar;
        ar.q = q;
        ar.q4 = 4 * q;
        ar.nq = 0 - q;
        ar.nq4 = 0 - 4 * q;
        ar.tw = nullptr;
        hipLaunchKernelGGL(calib_bfly_kernel<IntCal<true>>, dim3(blocks), dim3(256), 0, s, ar, buf, buf + 192,
                           iters);
      }
    }
    (void)hipEventRecord(e1, s);
    float ms = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0) {
      (void)hipGetLastError();
      set_error("calibration launch failed");
      rc = HELRM_EHIP;
    } else {
      *per_s = (double)threads * iters * 4 * 32 / (ms * 1e-3);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return rc;
}

int launch_ntt(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
               hipStream_t s) {
  return launch_ntt_epi(ctx, src, dst, ll, batch, forward, s, NttEpi{});
}

int launch_ntt_epi(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                   hipStream_t s, const NttEpi &epi) {
  if ((epi.a || epi.dup) && (!forward || epi.n_fin > HELRM_MAX_EPI || epi.n_fin > ll.n)) {
    set_error("NTT epilogue: forward transforms, finish on at most %d limbs", HELRM_MAX_EPI);
    return HELRM_EINVAL;
  }
  if (ctx->logn == 16) return launch_ntt_h<4>(ctx, src, dst, ll, batch, forward, s, epi);
  if (ctx->logn == 12) return launch_ntt_h<3>(ctx, src, dst, ll, batch, forward, s, epi);
  set_error("unsupported log_n %d (12 or 16)", ctx->logn);
  return HELRM_EINVAL;
}
