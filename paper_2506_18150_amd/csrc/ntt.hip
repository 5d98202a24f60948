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
// products; only the last pass reduces to [0,q).
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
template <int H, bool COLS>
struct Shape {
  static constexpr int E = 1 << H;                    // residues per thread
  static constexpr int R = E * E;                     // sub-transform length
  static constexpr int N = R * R;                     // ring degree
  static constexpr int W = COLS ? 16 : 8;             // sub-transforms per workgroup
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

// Forward stages on x[] in the "A" layout (element u + E k): global stage
// multiplier m = E/(2h), twiddle index m f + k/(2h).
template <int H>
__device__ __forceinline__ void fwd_phase_a(u64 (&x)[1 << H], const TW *tw, int f, u64 q) {
  constexpr int E = 1 << H;
  const u64 q2 = 2 * q;
#pragma unroll
  for (int h = E / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int k = 0; k < E; k++) {
      if ((k & h) == 0) {
        const TW t = tw[(E / (2 * h)) * f + k / (2 * h)];
        ct_bfly(x[k], x[k + h], t, q, q2);
      }
    }
  }
}

// Forward stages in the "B" layout (element E u + k): m = R/(2h), twiddle
// index m f + u E/(2h) + k/(2h).
template <int H>
__device__ __forceinline__ void fwd_phase_b(u64 (&x)[1 << H], const TW *tw, int f, int u, u64 q) {
  constexpr int E = 1 << H, R = E * E;
  const u64 q2 = 2 * q;
#pragma unroll
  for (int h = E / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int k = 0; k < E; k++) {
      if ((k & h) == 0) {
        const TW t = tw[(R / (2 * h)) * f + u * (E / (2 * h)) + k / (2 * h)];
        ct_bfly(x[k], x[k + h], t, q, q2);
      }
    }
  }
}

template <int H>
__device__ __forceinline__ void inv_phase_b(u64 (&x)[1 << H], const TW *tw, int f, int u, u64 q) {
  constexpr int E = 1 << H, R = E * E;
  const u64 q2 = 2 * q;
#pragma unroll
  for (int h = 1; h <= E / 2; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++) {
      if ((k & h) == 0) {
        const TW t = tw[(R / (2 * h)) * f + u * (E / (2 * h)) + k / (2 * h)];
        gs_bfly(x[k], x[k + h], t, q, q2);
      }
    }
  }
}

template <int H>
__device__ __forceinline__ void inv_phase_a(u64 (&x)[1 << H], const TW *tw, int f, u64 q) {
  constexpr int E = 1 << H;
  const u64 q2 = 2 * q;
#pragma unroll
  for (int h = 1; h <= E / 2; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++) {
      if ((k & h) == 0) {
        const TW t = tw[(E / (2 * h)) * f + k / (2 * h)];
        gs_bfly(x[k], x[k + h], t, q, q2);
      }
    }
  }
}

// One pass of the transform.  FWD: column pass first (src -> dst), block pass
// second (in place, final reduction).  INV: block pass first, column pass
// second (in place, times N^-1).
template <int H, bool FWD, bool COLS>
__global__ __launch_bounds__((Shape<H, COLS>::T)) void ntt_pass_kernel(const u64 *src, u64 *dst, LimbList ll,
                                                                     const TW *__restrict__ twtab,
                                                                     const PrimeInfo *__restrict__ pinfo,
                                                                     const NttEpi epi) {
  using S = Shape<H, COLS>;
  constexpr int E = S::E, R = S::R, N = S::N, W = S::W, WPL = S::WPL;
  __shared__ u64 lds[S::LDS];

  const int tid = threadIdx.x;
  const int limb_lin = blockIdx.x / WPL;
  const int part = blockIdx.x % WPL;
  const int bat = limb_lin / ll.n;
  const int li = limb_lin - bat * ll.n;
  const u64 *in = src + ((size_t)bat * ll.src_bstride + ll.src_off[li]) * (size_t)N;
  u64 *out = dst + ((size_t)bat * ll.dst_bstride + ll.dst_off[li]) * (size_t)N;
  const int p = ll.prime[li];
  const u64 q = pinfo[p].q;
  const TW *tw = twtab + (size_t)p * N;

  u64 x[E];
  if (COLS) {
    const int w = tid % W, u = tid / W;
    const int c = part * W + w;
    if (FWD) {
      // first forward pass: stages m = 1 .. R/2 on column c
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = in[c + R * (u + E * k)];
      fwd_phase_a<H>(x, tw, 1, q);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, u + E * k)] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = lds[col_idx<H, W>(w, E * u + k)];
      fwd_phase_b<H>(x, tw, 1, u, q);
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (E * u + k)] = x[k];
    } else {
      // last inverse pass: stages m = R/2 .. 1 on column c, then N^-1
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = in[c + R * (E * u + k)];
      inv_phase_b<H>(x, tw, 1, u, q);
#pragma unroll
      for (int k = 0; k < E; k++) lds[col_idx<H, W>(w, E * u + k)] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = lds[col_idx<H, W>(w, u + E * k)];
      inv_phase_a<H>(x, tw, 1, q);
      const u64 ni = pinfo[p].ninv, nip = pinfo[p].ninv_p;
#pragma unroll
      for (int k = 0; k < E; k++) out[c + R * (u + E * k)] = shoup(x[k], ni, nip, q);
    }
  } else {
    const int u = tid % E, w = tid / E;
    const int b = part * W + w;
    const int f = R + b;
    const u64 *ib = in + (size_t)R * b;
    u64 *ob = out + (size_t)R * b;
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = ib[u + E * k];
    if (FWD) {
      fwd_phase_a<H>(x, tw, f, q);
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = lds[blk_idx<H>(w, E * u + k)];
      fwd_phase_b<H>(x, tw, f, u, q);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = x[k];
      __syncthreads();
      const u64 q2 = 2 * q;
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
          u64 v = lds[blk_idx<H>(w, u + E * k)];
          v = v >= q2 ? v - q2 : v;
          v = v >= q ? v - q : v;
          eo[u + E * k] = shoup(sub_mod(ea[u + E * k], v, q), c.w, c.wp, q);
        }
      } else {
#pragma unroll
        for (int k = 0; k < E; k++) {
          u64 v = lds[blk_idx<H>(w, u + E * k)];
          v = v >= q2 ? v - q2 : v;
          v = v >= q ? v - q : v;
          ob[u + E * k] = v;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, u + E * k)] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = lds[blk_idx<H>(w, E * u + k)];
      inv_phase_b<H>(x, tw, f, u, q);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) lds[blk_idx<H>(w, E * u + k)] = x[k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = lds[blk_idx<H>(w, u + E * k)];
      inv_phase_a<H>(x, tw, f, q);
#pragma unroll
      for (int k = 0; k < E; k++) ob[u + E * k] = x[k];
    }
  }
}

template <int H>
int launch_ntt_h(helrm_ctx *ctx, const u64 *src, u64 *dst, const LimbList &ll, int batch, bool forward,
                 hipStream_t s, const NttEpi &epi) {
  using S = Shape<H, true>;
  using SC = Shape<H, true>;
  using SB = Shape<H, false>;
  LimbList second = ll;
  for (int i = 0; i < ll.n; i++) second.src_off[i] = ll.dst_off[i];
  second.src_bstride = ll.dst_bstride;
  const int gc = ll.n * batch * SC::WPL, gb = ll.n * batch * SB::WPL;
  if (gc == 0) return HELRM_OK;
  // per pass and limb: N words read and written, (N/2) log2(R) butterflies
  const double limbs = (double)ll.n * batch;
  const double bytes = limbs * 16.0 * S::N, ops = limbs * (S::N / 2) * (2 * H);
  KTimer tm(ctx, s);
  if (forward) {
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, true>), dim3(gc), dim3(SC::T), 0, s, src, dst, ll,
                       ctx->d_tw_fwd, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_FWD_COL, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, true, false>), dim3(gb), dim3(SB::T), 0, s, dst, dst,
                       second, ctx->d_tw_fwd, ctx->d_pinfo, epi);
    tm.lap(TK_NTT_FWD_BLK, epi.a ? bytes * 1.5 : bytes, ops);
  } else {
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, false>), dim3(gb), dim3(SB::T), 0, s, src, dst, ll,
                       ctx->d_tw_inv, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_INV_BLK, bytes, ops);
    hipLaunchKernelGGL((ntt_pass_kernel<H, false, true>), dim3(gc), dim3(SC::T), 0, s, dst, dst,
                       second, ctx->d_tw_inv, ctx->d_pinfo, NttEpi{});
    tm.lap(TK_NTT_INV_COL, bytes, ops);
  }
  HIP_TRY(hipGetLastError());
  return HELRM_OK;
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
