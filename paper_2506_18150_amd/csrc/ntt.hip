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
// consecutive lanes own consecutive elements.  Butterflies are Harvey's lazy
// ones (values in [0,4q) forward, [0,2q) inverse) with Shoup twiddle
// products for 60-bit primes and exact fp64 products for primes below 2^45;
// only the last pass reduces to [0,q).
#include "common.h"

namespace {

__device__ __forceinline__ void ct_bfly(u64 &x, u64 &y, const TW &t, u64 q, u64 q2) {
  u64 X = x >= q2 ? x - q2 : x;
  u64 T = shoup_lazy(y, t.w, t.wp, q);
  x = X + T;
  y = X - T + q2;
}

__device__ __forceinline__ void gs_bfly(u64 &x, u64 &y, const TW &t, u64 q, u64 q2) {
  u64 S = x + y;
  S = S >= q2 ? S - q2 : S;
  u64 D = x - y + q2;
  x = S;
  y = shoup_lazy(D, t.w, t.wp, q);
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
// IntA: residues as uint64 with Shoup twiddle products (any prime < 2^61).
// FltA: residues as fp64 for primes below 2^45, where every lazy value
// (< 4q < 2^47) and every twiddle is an exact double.  a*w mod q is computed
// exactly: h = fl(a w) and l = fma(a, w, -h) give a w = h + l exactly; the
// quotient estimate qq = floor(h * (1/q)) is off by at most one, so
// r = fma(-qq, q, h) + l (both steps exact) lies in (-q, 2q) and one
// correction brings it to [0, 2q).  fp64 FMA runs at full rate on gfx950,
// four times the rate of the 32-bit integer multiplies the Shoup product needs.

struct IntA {
  using V = u64;
  u64 q, q2;
  const TW *tw;
  __device__ __forceinline__ V load(u64 x) const { return x; }
  __device__ __forceinline__ u64 bits(V v) const { return v; }
  __device__ __forceinline__ V unbits(u64 b) const { return b; }
  __device__ __forceinline__ void ct(V &x, V &y, int idx) const { ct_bfly(x, y, tw[idx], q, q2); }
  __device__ __forceinline__ void gs(V &x, V &y, int idx) const { gs_bfly(x, y, tw[idx], q, q2); }
  // [0, 4q) -> [0, q)
  __device__ __forceinline__ u64 canon(V v) const {
    v = v >= q2 ? v - q2 : v;
    return v >= q ? v - q : v;
  }
  __device__ __forceinline__ u64 scale(V v, const PrimeInfo &pi) const { return shoup(v, pi.ninv, pi.ninv_p, q); }
};

struct FltA {
  using V = double;
  double q, q2, qinv;
  const double *tw;
  __device__ __forceinline__ V load(u64 x) const { return (double)x; }
  __device__ __forceinline__ u64 bits(V v) const { return (u64)__double_as_longlong(v); }
  __device__ __forceinline__ V unbits(u64 b) const { return __longlong_as_double((long long)b); }
  // a * w mod q in [0, 2q) for 0 <= a < 4q, 0 <= w < q
  __device__ __forceinline__ double mm(double a, double w) const {
#pragma clang fp contract(off)
    const double h = a * w;
    const double l = __fma_rn(a, w, -h);
    const double qq = floor(h * qinv);
    double r = __fma_rn(-qq, q, h) + l;
    return r < 0.0 ? r + q : r;
  }
  __device__ __forceinline__ void ct(V &x, V &y, int idx) const {
#pragma clang fp contract(off)
    const double X = x >= q2 ? x - q2 : x;
    const double T = mm(y, tw[idx]);
    x = X + T;
    y = (X - T) + q2;
  }
  __device__ __forceinline__ void gs(V &x, V &y, int idx) const {
#pragma clang fp contract(off)
    double S = x + y;
    S = S >= q2 ? S - q2 : S;
    const double D = (x - y) + q2;
    x = S;
    y = mm(D, tw[idx]);
  }
  __device__ __forceinline__ u64 canon(V v) const {
    v = v >= q2 ? v - q2 : v;
    v = v >= q ? v - q : v;
    return (u64)v;
  }
  __device__ __forceinline__ u64 scale(V v, const PrimeInfo &pi) const {
    double r = mm(v, pi.ninv_d);
    return (u64)(r >= q ? r - q : r);
  }
};

// Forward stages on x[] in the "A" layout (element u + E k): global stage
// multiplier m = E/(2h), twiddle index m f + k/(2h).
template <int H, class A>
__device__ __forceinline__ void fwd_phase_a(typename A::V (&x)[1 << H], const A &ar, int f) {
  constexpr int E = 1 << H;
#pragma unroll
  for (int h = E / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.ct(x[k], x[k + h], (E / (2 * h)) * f + k / (2 * h));
  }
}

// Forward stages in the "B" layout (element E u + k): m = R/(2h), twiddle
// index m f + u E/(2h) + k/(2h).
template <int H, class A>
__device__ __forceinline__ void fwd_phase_b(typename A::V (&x)[1 << H], const A &ar, int f, int u) {
  constexpr int E = 1 << H, R = E * E;
#pragma unroll
  for (int h = E / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.ct(x[k], x[k + h], (R / (2 * h)) * f + u * (E / (2 * h)) + k / (2 * h));
  }
}

template <int H, class A>
__device__ __forceinline__ void inv_phase_b(typename A::V (&x)[1 << H], const A &ar, int f, int u) {
  constexpr int E = 1 << H, R = E * E;
#pragma unroll
  for (int h = 1; h <= E / 2; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.gs(x[k], x[k + h], (R / (2 * h)) * f + u * (E / (2 * h)) + k / (2 * h));
  }
}

template <int H, class A>
__device__ __forceinline__ void inv_phase_a(typename A::V (&x)[1 << H], const A &ar, int f) {
  constexpr int E = 1 << H;
#pragma unroll
  for (int h = 1; h <= E / 2; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++)
      if ((k & h) == 0) ar.gs(x[k], x[k + h], (E / (2 * h)) * f + k / (2 * h));
  }
}

// The body of one pass for one arithmetic policy.
template <int H, bool FWD, bool COLS, int WS, class A>
__device__ __forceinline__ void pass_body(const A &ar, u64 *lds, const u64 *in, u64 *out, int part, int bat,
                                          int li, const PrimeInfo &pi, const NttEpi &epi) {
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
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.load(in[c + R * (u + E * k)]);
      fwd_phase_a<H>(x, ar, 1);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[col_idx<H, W>(w, E * u + k)]);
      fwd_phase_b<H>(x, ar, 1, u);
      // lazy values in [0, 4q) go to memory as integers
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (E * u + k)] = (u64)x[k];
    } else {
      // last inverse pass: stages m = R/2 .. 1 on column c, then N^-1
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.load(in[c + R * (E * u + k)]);
      inv_phase_b<H>(x, ar, 1, u);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[col_idx<H, W>(w, u + E * k)]);
      inv_phase_a<H>(x, ar, 1);
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (u + E * k)] = ar.scale(x[k], pi);
    }
  } else {
    const int u = tid % E, w = tid / E;
    const int b = part * W + w;
    const int f = R + b;
    const u64 *ib = in + (size_t)R * b;
    u64 *ob = out + (size_t)R * b;
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = ar.load(ib[u + E * k]);
    if (FWD) {
      fwd_phase_a<H>(x, ar, f);
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, E * u + k)]);
      fwd_phase_b<H>(x, ar, f, u);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
      const u64 q = pi.q;
      if (epi.a) {
        // fused finish: out = (a - NTT(x)) * c  (ModDown: c = P^-1, rescale: c = q_l^-1)
        const int bo = bat / epi.inner, bi = bat % epi.inner;
        const u64 *ea = epi.a + ((size_t)bo * epi.a_bs + (size_t)bi * epi.a_cs + epi.a_off[li]) * (size_t)N +
                        (size_t)R * b;
        u64 *eo = epi.out + ((size_t)bo * epi.out_bs + (size_t)bi * epi.out_cs + epi.out_off[li]) * (size_t)N +
                  (size_t)R * b;
        const TW c = epi.c[li];
#pragma unroll
        for (int k = 0; k < E; k++) {
          const u64 v = ar.canon(ar.unbits(lds[blk_idx<H>(w, u + E * k)]));
          eo[u + E * k] = shoup(sub_mod(ea[u + E * k], v, q), c.w, c.wp, q);
        }
      } else {
#pragma unroll
        for (int k = 0; k < E; k++) ob[u + E * k] = ar.canon(ar.unbits(lds[blk_idx<H>(w, u + E * k)]));
      }
    } else {
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, E * u + k)]);
      inv_phase_b<H>(x, ar, f, u);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = ar.bits(x[k]);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = ar.unbits(lds[blk_idx<H>(w, u + E * k)]);
      inv_phase_a<H>(x, ar, f);
      // values in [0, 2q) go to memory as integers
#pragma unroll
      for (int k = 0; k < E; k++) ob[u + E * k] = (u64)x[k];
    }
  }
}

// One pass of the transform.  FWD: column pass first (src -> dst), block pass
// second (in place, final reduction).  INV: block pass first, column pass
// second (in place, times N^-1).  Primes below 2^45 take the fp64 path.
template <int H, bool FWD, bool COLS, int WS>
__global__ __launch_bounds__((Shape<H, COLS, WS>::T)) void ntt_pass_kernel(const u64 *src, u64 *dst, LimbList ll,
                                                                         const TW *__restrict__ twtab,
                                                                         const double *__restrict__ twdtab,
                                                                         const PrimeInfo *__restrict__ pinfo,
                                                                         const NttEpi epi) {
  using S = Shape<H, COLS, WS>;
  constexpr int N = S::N, WPL = S::WPL;
  __shared__ u64 lds[S::LDS];
  const int limb_lin = blockIdx.x / WPL;
  const int part = blockIdx.x % WPL;
  const int bat = limb_lin / ll.n;
  const int li = limb_lin - bat * ll.n;
  const u64 *in = src + ((size_t)bat * ll.src_bstride + ll.src_off[li]) * (size_t)N;
  u64 *out = dst + ((size_t)bat * ll.dst_bstride + ll.dst_off[li]) * (size_t)N;
  const int p = ll.prime[li];
  const PrimeInfo pi = pinfo[p];
  if (pi.q < (1ull << 45)) {
    FltA ar{pi.qd, 2.0 * pi.qd, pi.qinv_d, twdtab + (size_t)p * N};
    pass_body<H, FWD, COLS, WS>(ar, lds, in, out, part, bat, li, pi, epi);
  } else {
    IntA ar{pi.q, 2 * pi.q, twtab + (size_t)p * N};
    pass_body<H, FWD, COLS, WS>(ar, lds, in, out, part, bat, li, pi, epi);
  }
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
  // per pass and limb: N words read and written, (N/2) log2(R) butterflies
  const double limbs = (double)ll.n * batch;
  const double bytes = limbs * 16.0 * SC::N, ops = limbs * (SC::N / 2) * (2 * H);
  KTimer tm(ctx, s);
  if (forward) {
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, true, WC>), dim3(gc), dim3(SC::T), 0, s, src, dst, ll,
                       ctx->d_tw_fwd, ctx->d_twd_fwd, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_FWD_COL, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, false, WB>), dim3(gb), dim3(SB::T), 0, s, dst, dst,
                       second, ctx->d_tw_fwd, ctx->d_twd_fwd, ctx->d_pinfo, epi);
    tm.lap(TK_NTT_FWD_BLK, epi.a ? bytes * 1.5 : bytes, ops);
  } else {
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, false, WB>), dim3(gb), dim3(SB::T), 0, s, src, dst, ll,
                       ctx->d_tw_inv, ctx->d_twd_inv, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_INV_BLK, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, true, WC>), dim3(gc), dim3(SC::T), 0, s, dst, dst,
                       second, ctx->d_tw_inv, ctx->d_twd_inv, ctx->d_pinfo, NttEpi{});
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

}  // namespace

int launch_ntt(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
               hipStream_t s) {
  return launch_ntt_epi(ctx, src, dst, ll, batch, forward, s, NttEpi{});
}

int launch_ntt_epi(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                   hipStream_t s, const NttEpi &epi) {
  if (epi.a && (!forward || ll.n > HELRM_MAX_EPI)) {
    set_error("NTT epilogue: forward transforms of at most %d limbs only", HELRM_MAX_EPI);
    return HELRM_EINVAL;
  }
  if (ctx->logn == 16) return launch_ntt_h<4>(ctx, src, dst, ll, batch, forward, s, epi);
  if (ctx->logn == 12) return launch_ntt_h<3>(ctx, src, dst, ll, batch, forward, s, epi);
  set_error("unsupported log_n %d (12 or 16)", ctx->logn);
  return HELRM_EINVAL;
}
