// C ABI of libhelrm: context set-up (roots, twiddles, conversion constants),
// resident evaluation keys and plans, and the host orchestration of the
// key-switching, rescale and double-hoisted BSGS matvec pipelines.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "common.h"

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

extern "C" const char *helrm_last_error(void) { return g_last_error.c_str(); }

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                          \
  }                                                            \
  catch (const std::bad_alloc &) {                             \
    set_error("host allocation failed");                       \
    return HELRM_ENOMEM;                                       \
  }                                                            \
  catch (...) {                                                \
    set_error("internal error");                               \
    return HELRM_ESTATE;                                       \
  }

// ---------------------------------------------------------------- kernel timing

hipEvent_t timing_event(helrm_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->tmu);
  if (!ctx->evpool.empty()) {
    hipEvent_t e = ctx->evpool.back();
    ctx->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void timing_push(helrm_ctx *ctx, int k, hipEvent_t a, hipEvent_t b, double bytes, double ops) {
  std::lock_guard<std::mutex> lk(ctx->tmu);
  ctx->trecs.push_back(TimingRec{k, a, b, bytes, ops});
}

static const char *const kTimedNames[TK_COUNT] = {"ntt_fwd_col", "ntt_fwd_blk", "ntt_inv_blk", "ntt_inv_col",
                                                  "conv",        "ks_acc",      "baby_mac",    "sub_mul",
                                                  "baby_mfma",   "baby_fold"};

static void timing_clear(helrm_ctx *ctx) {
  std::vector<hipEvent_t> seen;
  for (auto &r : ctx->trecs) {
    seen.push_back(r.a);
    seen.push_back(r.b);
  }
  std::sort(seen.begin(), seen.end());
  seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
  for (auto e : seen) ctx->evpool.push_back(e);
  ctx->trecs.clear();
}

// ---------------------------------------------------------------- host modular arithmetic

namespace {

u64 hmul(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 hpow(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = hmul(r, a, q);
    a = hmul(a, a, q);
    e >>= 1;
  }
  return r;
}

// inverse modulo q (q odd, gcd(a, q) = 1) by the extended Euclidean algorithm
u64 hinv(u64 a, u64 q) {
  __int128 t = 0, nt = 1, r = q, nr = a % q;
  while (nr != 0) {
    __int128 qq = r / nr, tmp;
    tmp = t - qq * nt; t = nt; nt = tmp;
    tmp = r - qq * nr; r = nr; nr = tmp;
  }
  if (t < 0) t += q;
  return (u64)t;
}

u64 shoup_of(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

TW tw_of(u64 w, u64 q) { return TW{w % q, shoup_of(w % q, q)}; }

u64 neg_inv64(u64 q) {
  u64 x = q;  // q * q = 1 mod 8 for odd q
  for (int i = 0; i < 6; i++) x *= 2 - q * x;
  return (u64)0 - x;
}

u64 mont_of(u64 w, u64 q) { return (u64)(((u128)(w % q) << 64) % q); }

unsigned brv(unsigned x, int bits) {
  unsigned r = 0;
  for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

// ---------------------------------------------------------------- constant buffer builder

struct ConstBuilder {
  std::vector<u64> words;
  size_t add_tw(const std::vector<TW> &v) {
    size_t off = words.size();
    for (auto &t : v) { words.push_back(t.w); words.push_back(t.wp); }
    return off;
  }
  size_t add_u64(const std::vector<u64> &v) {
    size_t off = words.size();
    words.insert(words.end(), v.begin(), v.end());
    return off;
  }
};

// Fast base conversion constants from input primes to output primes.
void build_conv(helrm_ctx *c, ConstBuilder &cb, const std::vector<int> &in, const std::vector<int> &out,
                ConvTable &t, size_t &off_inv, size_t &off_mont) {
  t.nin = (int)in.size();
  t.nout = (int)out.size();
  for (int i = 0; i < t.nin; i++) t.in_prime[i] = in[i];
  for (int r = 0; r < t.nout; r++) t.out_prime[r] = out[r];
  std::vector<TW> inv(t.nin);
  std::vector<u64> mont((size_t)t.nin * t.nout);
  for (int i = 0; i < t.nin; i++) {
    const u64 qi = c->primes[in[i]];
    u64 hat = 1;  // (Qin / q_i) mod q_i
    for (int k = 0; k < t.nin; k++)
      if (k != i) hat = hmul(hat, c->primes[in[k]] % qi, qi);
    inv[i] = tw_of(hinv(hat, qi), qi);
    for (int r = 0; r < t.nout; r++) {
      const u64 qr = c->primes[out[r]];
      u64 h = 1;  // (Qin / q_i) mod r
      for (int k = 0; k < t.nin; k++)
        if (k != i) h = hmul(h, c->primes[in[k]] % qr, qr);
      mont[(size_t)i * t.nout + r] = mont_of(h, qr);
    }
  }
  off_inv = cb.add_tw(inv);
  off_mont = cb.add_u64(mont);
}

// ---------------------------------------------------------------- workspace

struct Arena {
  char *base;
  size_t used = 0;
  u64 *take(size_t words) {
    u64 *p = (u64 *)(base + used);
    used += ((words * sizeof(u64) + 255) / 256) * 256;
    return p;
  }
};

// The workspace of stream s, grown to at least `bytes`.  Growing is refused
// while s is being captured (the graph would record an allocation); a
// workspace a capture has used is never freed when it is outgrown, only
// retired until helrm_destroy, so graphs captured on it stay valid.
int ensure_ws(helrm_ctx *ctx, hipStream_t s, size_t bytes, char **out) {
  std::lock_guard<std::mutex> lk(ctx->ws_mu);
  Workspace &w = ctx->ws[s];
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    cs = hipStreamCaptureStatusNone;
  }
  const bool capturing = cs != hipStreamCaptureStatusNone;
  if (w.bytes < bytes) {
    if (capturing) {
      set_error("the stream's workspace holds %zu bytes and this call needs %zu: reserve it before capturing "
                "(helrm_reserve / helrm_reserve_multi)", w.bytes, bytes);
      return HELRM_ESTATE;
    }
    if (w.ptr) {
      if (w.captured) {
        ctx->ws_retired.push_back(w.ptr);
      } else {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(w.ptr));
      }
      w.ptr = nullptr;
      w.bytes = 0;
      w.captured = false;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("workspace allocation of %zu bytes failed", bytes);
      return HELRM_ENOMEM;
    }
    w.ptr = p;
    w.bytes = bytes;
  }
  if (capturing) w.captured = true;
  *out = (char *)w.ptr;
  return HELRM_OK;
}

size_t rnd(size_t words) { return ((words * sizeof(u64) + 255) / 256) * 256; }

}  // namespace

// Static scratch of helrm_lookup_packed_noalloc: one array per device, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it only names the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device, resolved once per
// device when a context is created on it.
static __device__ __align__(256) unsigned char scratch[HELRM_NOALLOC_MAX_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_addr;   // device -> address of that device's `scratch`

// Device address of `scratch` on `dev`, which must be the current device.
int scratch_address(int dev, char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return HELRM_OK;
  }
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    set_error("hipGetSymbolAddress of the static scratch failed on device %d: %s", dev, hipGetErrorString(e));
    return HELRM_EHIP;
  }
  g_scratch_addr[dev] = (char *)ptr;
  *out = (char *)ptr;
  return HELRM_OK;
}

// ---------------------------------------------------------------- limb lists

LimbList ll_make(int n, int src_bs, int dst_bs) {
  LimbList ll;
  memset(&ll, 0, sizeof ll);
  ll.n = n;
  ll.src_bstride = src_bs;
  ll.dst_bstride = dst_bs;
  return ll;
}

// ---------------------------------------------------------------- pipeline pieces

// ModUp of c1 (evaluation form, [level+1] limbs, batch stride c1_bs limbs) to
// digits D ([beta][pqn] limbs per batch element, stride d_bs limbs).
int do_modup(helrm_ctx *ctx, int level, const u64 *c1, int c1_bs, u64 *D, int d_bs, u64 *coef, int batch,
             hipStream_t s) {
  const int N = ctx->N, qn = level + 1, pqn = level + 1 + ctx->K, beta = ctx->n_digits(level);
  // 1. coefficient form of c1
  LimbList a = ll_make(qn, c1_bs, qn);
  for (int i = 0; i < qn; i++) { a.src_off[i] = i; a.dst_off[i] = i; a.prime[i] = (unsigned char)i; }
  TRY(launch_ntt(ctx, c1, coef, a, batch, false, s));
  // 2. base conversion of every digit to the other primes of PQ_level; the
  //    digit's own limbs are c1's limbs (copied in evaluation form)
  LimbList nt = ll_make(0, d_bs, d_bs);
  ConvSpec specs[HELRM_MAX_CONV_JOBS];
  CHECK_ARG(beta <= HELRM_MAX_CONV_JOBS, "modup: at most %d digits", HELRM_MAX_CONV_JOBS);
  for (int j = 0; j < beta; j++) {
    ConvSpec &sp = specs[j];
    sp.t = &ctx->modup_tabs[level][j];
    const int lo = ctx->digit_lo(j), hi = ctx->digit_hi(j, level);
    sp.src_off0 = lo;
    int k = 0;
    for (int r = 0; r < pqn; r++) {
      if (r >= lo && r < hi) continue;
      sp.dst_off[k++] = j * pqn + r;
      if (nt.n >= HELRM_MAX_LIMBS) { set_error("modup: too many limbs"); return HELRM_EINVAL; }
      nt.src_off[nt.n] = j * pqn + r;
      nt.dst_off[nt.n] = j * pqn + r;
      nt.prime[nt.n] = (unsigned char)ctx->pq_prime(r, level);
      nt.n++;
    }
    sp.ncopy = hi - lo;
    for (int i = lo; i < hi; i++) {
      sp.copy_src_off[i - lo] = i;
      sp.copy_dst_off[i - lo] = j * pqn + i;
    }
  }
  TRY(launch_conv(ctx, specs, beta, coef, qn, c1, c1_bs, D, d_bs, batch, s));
  // 3. back to evaluation form
  TRY(launch_ntt(ctx, D, D, nt, batch, true, s));
  return HELRM_OK;
}

// ModDown of X ([2][pqn] limbs per element, stride x_bs) to out ([2][qn],
// stride out_bs).  mdP: [2K] limbs per element, mdT: [2 qn] per element.
int do_moddown(helrm_ctx *ctx, int level, const u64 *X, int x_bs, u64 *out, int out_bs, u64 *mdP, u64 *mdT,
               int batch, hipStream_t s) {
  const int K = ctx->K, qn = level + 1, pqn = level + 1 + K;
  // 1. special limbs to coefficient form
  LimbList a = ll_make(2 * K, x_bs, 2 * K);
  for (int c = 0; c < 2; c++)
    for (int k = 0; k < K; k++) {
      a.src_off[c * K + k] = c * pqn + qn + k;
      a.dst_off[c * K + k] = c * K + k;
      a.prime[c * K + k] = (unsigned char)(ctx->L + 1 + k);
    }
  TRY(launch_ntt(ctx, X, mdP, a, batch, false, s));
  // 2. convert P -> Q_level (both polynomials as a batch of 2*batch)
  ConvSpec sp;
  sp.t = &ctx->moddown_tabs[level];
  sp.src_off0 = 0;
  for (int i = 0; i < qn; i++) sp.dst_off[i] = i;
  sp.ncopy = 0;
  TRY(launch_conv(ctx, &sp, 1, mdP, K, nullptr, 0, mdT, qn, 2 * batch, s));
  // 3. evaluation form, fused with 4. out_i = (X_i - t_i) P^-1
  LimbList b = ll_make(qn, qn, qn);
  for (int i = 0; i < qn; i++) { b.src_off[i] = i; b.dst_off[i] = i; b.prime[i] = (unsigned char)i; }
  NttEpi e;
  e.a = X;
  e.out = out;
  e.c = ctx->moddown_pinv[level];
  e.inner = 2;
  e.n_fin = qn;
  e.a_bs = x_bs;
  e.a_cs = pqn;
  e.out_bs = out_bs;
  e.out_cs = qn;
  for (int i = 0; i < qn; i++) { e.a_off[i] = i; e.out_off[i] = i; }
  TRY(launch_ntt_epi(ctx, mdT, mdT, b, 2 * batch, true, s, e));
  return HELRM_OK;
}

int do_rescale(helrm_ctx *ctx, int level, const u64 *in, int in_bs, u64 *out, int out_bs, u64 *top, u64 *V,
               int batch, hipStream_t s) {
  const int qn = level + 1;
  LimbList a = ll_make(2, in_bs, 2);
  for (int c = 0; c < 2; c++) {
    a.src_off[c] = c * qn + level;
    a.dst_off[c] = c;
    a.prime[c] = (unsigned char)level;
  }
  TRY(launch_ntt(ctx, in, top, a, batch, false, s));
  TRY(launch_rescale_spread(ctx, top, V, level, batch, s));
  LimbList b = ll_make(level, level, level);
  for (int i = 0; i < level; i++) { b.src_off[i] = i; b.dst_off[i] = i; b.prime[i] = (unsigned char)i; }
  // evaluation form fused with out_i = (c_i - v_i) q_l^-1
  NttEpi e;
  e.a = in;
  e.out = out;
  e.c = ctx->rescale_qinv[level];
  e.inner = 2;
  e.n_fin = level;
  e.a_bs = in_bs;
  e.a_cs = qn;
  e.out_bs = out_bs;
  e.out_cs = level;
  for (int i = 0; i < level; i++) { e.a_off[i] = i; e.out_off[i] = i; }
  TRY(launch_ntt_epi(ctx, V, V, b, 2 * batch, true, s, e));
  return HELRM_OK;
}

// A ModDown whose result feeds a ModUp (the next key switch of a fold or
// giant step), done in coefficient form: NTT^-1 is exact and linear, so
// (X - NTT(t)) P^-1 in evaluation form and NTT((NTT^-1(X) - t) P^-1) are the
// same residues, and the ModUp's own NTT^-1 of c1 disappears.
//   1. NTT^-1 of c0's special limbs and of all of c1's limbs (X -> C);
//   2. one conversion P -> Q: t0 for c0, z1 = (X1 - t1) P^-1 for c1 (C -> F);
//   3. the ModUp conversion of z1 to every digit (F -> F);
//   4. one forward NTT of t0 (finished into z.c0: (X0 - NTT(t0)) P^-1), of z1
//      (into the digits' own limbs and z.c1) and of the converted limbs.
// X: [batch] x x_bs limbs, (c0, c1) PQ limbs at 0 and pqn; z: [batch][2][qn]
// at batch stride z_bs; F: [batch] x f_bs limbs, t0 at 0, z1 at qn, digits
// ([beta][pqn]) at 2 qn; C: [batch][K + pqn].
int fused_fits(const helrm_ctx *ctx, int level) {
  const int qn = level + 1, pqn = level + 1 + ctx->K;
  return 2 * qn + ctx->n_digits(level) * pqn - qn <= HELRM_MAX_LIMBS && ctx->K + pqn <= HELRM_MAX_LIMBS &&
         2 * pqn <= HELRM_MAX_LIMBS && qn <= HELRM_MAX_EPI;
}

int do_moddown_modup(helrm_ctx *ctx, int level, const u64 *X, int x_bs, u64 *z, int z_bs, u64 *F, int f_bs,
                     u64 *C, int batch, hipStream_t s) {
  const int K = ctx->K, qn = level + 1, pqn = level + 1 + K, beta = ctx->n_digits(level);
  const int c_bs = K + pqn;
  CHECK_ARG(beta <= HELRM_MAX_CONV_JOBS, "modup: at most %d digits", HELRM_MAX_CONV_JOBS);
  // 1.
  LimbList a = ll_make(K + pqn, x_bs, c_bs);
  for (int k = 0; k < K; k++) {
    a.src_off[k] = qn + k;
    a.dst_off[k] = k;
    a.prime[k] = ctx->L + 1 + k;
  }
  for (int i = 0; i < pqn; i++) {
    a.src_off[K + i] = pqn + i;
    a.dst_off[K + i] = K + i;
    a.prime[K + i] = ctx->pq_prime(i, level);
  }
  TRY(launch_ntt(ctx, X, C, a, batch, false, s));
  // 2.  With digits of at most K limbs, the ModDown of c1 runs in front of
  // each digit's ModUp conversion (step 3), in one launch with t0's conversion
  bool fuse = ctx->tune_fuse_conv && beta + 1 <= HELRM_MAX_CONV_JOBS && ctx->moddown_tabs[level].nin == K;
  for (int j = 0; j < beta; j++) fuse = fuse && ctx->digit_hi(j, level) - ctx->digit_lo(j) <= K;
  ConvSpec md[2];
  for (int c = 0; c < 2; c++) {
    md[c].t = &ctx->moddown_tabs[level];
    md[c].src_off0 = c == 0 ? 0 : K + qn;
    for (int i = 0; i < qn; i++) md[c].dst_off[i] = c * qn + i;
  }
  md[1].fin = CONV_FIN_MODDOWN;
  md[1].fin_off0 = K;
  // 3.
  ConvSpec up[HELRM_MAX_CONV_JOBS];
  LimbList f = ll_make(0, f_bs, f_bs);
  NttEpi e;
  e.a = X;
  e.out = z;
  e.c = ctx->moddown_pinv[level];
  e.inner = 1;
  e.n_fin = qn;
  e.a_bs = x_bs;
  e.out_bs = z_bs;
  e.dup = z;
  e.dup_bs = z_bs;
  for (int i = 0; i < qn; i++) {   // t0 -> z.c0 (finish)
    f.src_off[f.n] = i;
    f.dst_off[f.n] = i;
    f.prime[f.n] = i;
    e.a_off[i] = i;
    e.out_off[i] = i;
    e.dup_off[f.n] = -1;
    f.n++;
  }
  for (int j = 0; j < beta; j++) {
    const int lo = ctx->digit_lo(j), hi = ctx->digit_hi(j, level);
    for (int i = lo; i < hi; i++) {   // z1 -> digit j's own limb and z.c1
      f.src_off[f.n] = qn + i;
      f.dst_off[f.n] = 2 * qn + j * pqn + i;
      f.prime[f.n] = i;
      e.dup_off[f.n] = qn + i;
      f.n++;
    }
  }
  for (int j = 0; j < beta; j++) {
    ConvSpec &sp = up[fuse ? j + 1 : j];
    sp.t = &ctx->modup_tabs[level][j];
    const int lo = ctx->digit_lo(j), hi = ctx->digit_hi(j, level);
    sp.src_off0 = qn + lo;
    if (fuse) {   // inputs z1 on the digit's limbs, formed from C and written to F
      sp.pre = &ctx->moddown_tabs[level];
      sp.pre_src0 = K + qn;
      sp.pre_a0 = K + lo;
      sp.pre_col0 = lo;
      sp.pre_dst0 = qn + lo;
    }
    int k = 0;
    for (int r = 0; r < pqn; r++) {
      if (r >= lo && r < hi) continue;
      sp.dst_off[k++] = 2 * qn + j * pqn + r;
      f.src_off[f.n] = 2 * qn + j * pqn + r;
      f.dst_off[f.n] = 2 * qn + j * pqn + r;
      f.prime[f.n] = ctx->pq_prime(r, level);
      e.dup_off[f.n] = -1;
      f.n++;
    }
  }
  if (fuse) {
    up[0] = md[0];
    TRY(launch_conv(ctx, up, beta + 1, C, c_bs, nullptr, 0, F, f_bs, batch, s));
  } else {
    TRY(launch_conv(ctx, md, 2, C, c_bs, nullptr, 0, F, f_bs, batch, s));
    TRY(launch_conv(ctx, up, beta, F, f_bs, nullptr, 0, F, f_bs, batch, s));
  }
  // 4.
  TRY(launch_ntt_epi(ctx, F, F, f, batch, true, s, e));
  return HELRM_OK;
}

// A ModDown followed by the rescale by q_level, in coefficient form:
// NTT^-1 of every limb of X (-> C), one conversion P -> Q_level with both
// finishes (-> F as [batch][2][level] coefficient limbs), one forward NTT
// (-> out, [batch][2][level] at batch stride out_bs).
int do_moddown_rescale(helrm_ctx *ctx, int level, const u64 *X, int x_bs, u64 *out, int out_bs, u64 *F,
                       u64 *C, int batch, hipStream_t s) {
  const int K = ctx->K, qn = level + 1, pqn = level + 1 + K;
  LimbList a = ll_make(2 * pqn, x_bs, 2 * pqn);
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < pqn; i++) {
      a.src_off[c * pqn + i] = c * pqn + i;
      a.dst_off[c * pqn + i] = c * pqn + i;
      a.prime[c * pqn + i] = ctx->pq_prime(i, level);
    }
  TRY(launch_ntt(ctx, X, C, a, batch, false, s));
  ConvSpec md[2];
  for (int c = 0; c < 2; c++) {
    md[c].t = &ctx->moddown_tabs[level];
    md[c].src_off0 = c * pqn + qn;
    md[c].fin = CONV_FIN_RESCALE;
    md[c].fin_off0 = c * pqn;
    md[c].qlinv = ctx->rescale_qinv[level];
    for (int i = 0; i < level; i++) md[c].dst_off[i] = c * level + i;
  }
  TRY(launch_conv(ctx, md, 2, C, 2 * pqn, nullptr, 0, F, 2 * level, batch, s));
  LimbList b = ll_make(2 * level, 2 * level, out_bs);
  for (int c = 0; c < 2; c++)
    for (int i = 0; i < level; i++) {
      b.src_off[c * level + i] = c * level + i;
      b.dst_off[c * level + i] = c * level + i;
      b.prime[c * level + i] = i;
    }
  TRY(launch_ntt(ctx, F, out, b, batch, true, s));
  return HELRM_OK;
}

// Key, Galois element and seed of the rotation by `step` into t.
int key_for(helrm_ctx *ctx, long step, KsTerm *t) {
  t->galois = galois_of_step(ctx, step);
  auto it = ctx->keys.find(t->galois);
  if (it == ctx->keys.end()) {
    set_error("no evaluation key loaded for rotation %ld (galois %u)", step, t->galois);
    return HELRM_EINVAL;
  }
  t->key = it->second.d;
  t->seed = it->second.seed;
  t->seeded = it->second.seeded;
  return HELRM_OK;
}

// workspace words of one ModUp + ModDown at this level and batch
struct KsSizes {
  size_t coef, D, X, mdP, mdT;
};

KsSizes ks_sizes(const helrm_ctx *ctx, int level, int batch, int n_pq) {
  const size_t N = ctx->N, qn = level + 1, pqn = level + 1 + ctx->K, beta = ctx->n_digits(level);
  KsSizes z;
  z.coef = batch * qn * N;
  z.D = batch * beta * pqn * N;
  z.X = (size_t)batch * n_pq * 2 * pqn * N;
  z.mdP = (size_t)batch * n_pq * 2 * ctx->K * N;
  z.mdT = (size_t)batch * n_pq * 2 * qn * N;
  return z;
}

// ---------------------------------------------------------------- matvec

// F: per batch element [t0: qn][z1: qn][digits: beta][pqn] (do_moddown_modup);
// the digits of every ModUp of the path live in F at offset 2 qn.
// C: coefficient-form limbs of a ModDown input ([2][pqn] per element).
struct MatvecWS {
  u64 *coef, *F, *C, *Dg, *X, *xg, *acc, *zA, *zB, *mdP, *mdT, *top, *V, *mv;
  uint32_t *E;   // entries of the key-folded product (plans with folded operands), or null
};

// Non-zero giant steps of a plan, or of the union of several plans' giants.
size_t nonzero_giants(const helrm_plan *const *ps, int n_in) {
  std::vector<int> u;
  for (int c = 0; c < n_in; c++)
    for (int g : ps[c]->giants)
      if (g != 0 && std::find(u.begin(), u.end(), g) == u.end()) u.push_back(g);
  return u.size();
}

size_t matvec_ws_bytes(const helrm_ctx *ctx, const helrm_plan *p, int batch, bool with_rescale,
                       size_t ng_union = 0) {
  const size_t N = ctx->N, lv = p->level, qn = lv + 1, pqn = lv + 1 + ctx->K, beta = ctx->n_digits((int)lv);
  const size_t B = batch, n2 = p->n2;
  const size_t ng = std::max(ng_union, nonzero_giants(&p, 1));
  size_t tot = 0;
  tot += rnd(B * n2 * qn * N);                  // coef (one ModUp of every giant's x_g)
  tot += rnd(B * (2 * qn + beta * pqn) * N);    // F
  tot += rnd(B * 2 * pqn * N);                  // C
  tot += rnd(B * (ng > 0 ? n2 : 1) * beta * pqn * N);  // Dg
  tot += rnd(B * n2 * 2 * pqn * N);             // X
  tot += rnd(B * n2 * 2 * qn * N);              // xg
  tot += rnd(B * 2 * pqn * N);                  // acc
  tot += 2 * rnd(B * 2 * qn * N);               // zA, zB
  tot += rnd(B * n2 * 2 * ctx->K * N);          // mdP
  tot += rnd(B * n2 * 2 * qn * N);              // mdT
  if (with_rescale) {
    tot += rnd(B * 2 * N);                      // top
    tot += rnd(B * 2 * lv * N);                 // V
    tot += rnd(B * 2 * qn * N);                 // matvec result
  }
  if (p->d_wm) tot += rnd(B * fold_entry_words(ctx, (int)lv) / 2);   // E (32-bit words)
  return tot;
}

MatvecWS carve_matvec(const helrm_ctx *ctx, const helrm_plan *p, int batch, bool with_rescale, char *base,
                      size_t ng_union = 0) {
  const size_t N = ctx->N, lv = p->level, qn = lv + 1, pqn = lv + 1 + ctx->K, beta = ctx->n_digits((int)lv);
  const size_t B = batch, n2 = p->n2;
  const size_t ng = std::max(ng_union, nonzero_giants(&p, 1));
  Arena a{base};
  MatvecWS w;
  w.coef = a.take(B * n2 * qn * N);
  w.F = a.take(B * (2 * qn + beta * pqn) * N);
  w.C = a.take(B * 2 * pqn * N);
  w.Dg = a.take(B * (ng > 0 ? n2 : 1) * beta * pqn * N);
  w.X = a.take(B * n2 * 2 * pqn * N);
  w.xg = a.take(B * n2 * 2 * qn * N);
  w.acc = a.take(B * 2 * pqn * N);
  w.zA = a.take(B * 2 * qn * N);
  w.zB = a.take(B * 2 * qn * N);
  w.mdP = a.take(B * n2 * 2 * ctx->K * N);
  w.mdT = a.take(B * n2 * 2 * qn * N);
  w.top = w.V = w.mv = nullptr;
  if (with_rescale) {
    w.top = a.take(B * 2 * N);
    w.V = a.take(B * 2 * lv * N);
    w.mv = a.take(B * 2 * qn * N);
  }
  w.E = p->d_wm ? (uint32_t *)a.take(B * fold_entry_words(ctx, (int)lv) / 2) : nullptr;
  return w;
}

// Matvec of n_in ciphertexts (the column blocks of one selector) with plans
// that share m, n1, n2 and the fold; ciphertext c of batch element b is at
// ct + (b * ct_bs + 2 (level+1) c) limbs.  Every block's baby-step products
// go into the same giant accumulators X_g, then ModDown, giant steps and the
// fold run once.  The result (level `level`) goes to out; with rs_out, the
// rescaled result (level - 1, [batch][2][level]) goes to rs_out.  A ModDown
// that feeds a ModUp or the rescale runs fused with it in coefficient form
// (knob fuse_ks).
int run_matvec(helrm_ctx *ctx, const helrm_plan *const *ps, int n_in, const u64 *ct, int ct_bs, u64 *out,
               u64 *rs_out, int batch, MatvecWS &w, hipStream_t s) {
  const helrm_plan *p = ps[0];
  const int N = ctx->N, lv = p->level, qn = lv + 1, pqn = lv + 1 + ctx->K, beta = ctx->n_digits(lv);
  const int n2 = p->n2;
  const int d_bs = beta * pqn;               // Dg: [giant][beta][pqn] per element
  const int f_bs = 2 * qn + beta * pqn;      // F
  u64 *const D = w.F + (size_t)2 * qn * N;   // digits in F
  const size_t x_bs = (size_t)n2 * 2 * pqn;  // limbs per batch element of X
  const bool fuse = ctx->tune_fuse_ks && fused_fits(ctx, lv);
  std::vector<int> giants;
  for (int c = 0; c < n_in; c++) {
    const helrm_plan *pc = ps[c];
    const u64 *ctc = ct + (size_t)c * 2 * qn * N;
    // 1. hoisted ModUp of c1
    TRY(do_modup(ctx, lv, ctc + (size_t)qn * N, ct_bs, D, f_bs, w.coef, batch, s));
    // 2. fused baby steps + plaintext MAC, giant outputs in tiles (the first
    //    block writes every tile a later block may add to)
    for (int g0 = 0; g0 < n2; g0 += HELRM_MAX_GTILE) {
      const int ng = std::min(HELRM_MAX_GTILE, n2 - g0);
      bool any = false;
      for (int g : pc->giants)
        if (g >= g0 && g < g0 + ng) any = true;
      const bool force = c == 0 && n_in > 1;
      if (!any && !force) continue;
      TRY(launch_baby_mac(ctx, pc, D, (size_t)f_bs * N, ctc, (size_t)ct_bs * N, w.X + (size_t)g0 * 2 * pqn * N,
                          x_bs * N, g0, ng, batch, s, c > 0, force, pc->d_wm ? w.E : nullptr));
    }
    for (int g : pc->giants)
      if (std::find(giants.begin(), giants.end(), g) == giants.end()) giants.push_back(g);
  }
  std::sort(giants.begin(), giants.end());
  const bool only0 = giants.size() == 1 && giants[0] == 0;
  const bool no_fold = p->stages.empty();
  bool z_digits = false;   // D holds the ModUp of the current z's c1
  const u64 *z = nullptr;
  if (only0 && fuse) {
    // 3. x_0 = ModDown(X_0), fused with what follows it
    if (no_fold) {
      if (rs_out) {
        TRY(do_moddown_rescale(ctx, lv, w.X, (int)x_bs, rs_out, 2 * lv, w.F, w.C, batch, s));
        return HELRM_OK;
      }
      return do_moddown(ctx, lv, w.X, (int)x_bs, out, 2 * qn, w.mdP, w.mdT, batch, s);
    }
    TRY(do_moddown_modup(ctx, lv, w.X, (int)x_bs, w.zA, 2 * qn, w.F, f_bs, w.C, batch, s));
    z = w.zA;
    z_digits = true;
  } else {
    // 3. x_g = ModDown(X_g) for every g (batch of batch*n2)
    TRY(do_moddown(ctx, lv, w.X, 2 * pqn, w.xg, 2 * qn, w.mdP, w.mdT, batch * n2, s));
    u64 *zbuf = w.zA;
    if (only0) {
      if (no_fold) {
        // copy x_0 to out
        LimbList cp = ll_make(2 * qn, n2 * 2 * qn, 2 * qn);
        for (int i = 0; i < 2 * qn; i++) { cp.src_off[i] = i; cp.dst_off[i] = i; cp.prime[i] = 0; }
        TRY(launch_copy_limbs(w.xg, out, cp, batch, N, s));
      } else if (n2 == 1) {
        // x_0 is element 0 of every n2-group of xg; with one giant step xg
        // already has the layout of z
        z = w.xg;
      } else {
        LimbList cp = ll_make(2 * qn, n2 * 2 * qn, 2 * qn);
        for (int i = 0; i < 2 * qn; i++) { cp.src_off[i] = i; cp.dst_off[i] = i; cp.prime[i] = 0; }
        TRY(launch_copy_limbs(w.xg, zbuf, cp, batch, N, s));
        z = zbuf;
      }
    } else {
      // 4. giant rotations by n1 g of x_g (g >= 1), accumulated in PQ with P
      //    x_0: one ModUp covers every x_g of the batch (batch * n2
      //    ciphertexts, x_0's digits unused), so its launches do not repeat
      //    per giant step
      TRY(do_modup(ctx, lv, w.xg + (size_t)qn * N, 2 * qn, w.Dg, d_bs, w.coef, batch * n2, s));
      std::vector<KsTerm> terms;
      for (int g : giants) {
        if (g == 0) continue;
        KsTerm t;
        t.digits = w.Dg + (size_t)g * d_bs * N;
        t.c0 = w.xg + (size_t)g * 2 * qn * N;
        TRY(key_for(ctx, (long)p->sign * p->n1 * g, &t));
        terms.push_back(t);
      }
      const bool has0 = giants[0] == 0;
      TRY(launch_ks_accumulate(ctx, lv, terms.data(), (int)terms.size(), (size_t)n2 * d_bs * N,
                               (size_t)n2 * 2 * qn * N, has0 ? w.xg : nullptr, (size_t)n2 * 2 * qn * N, w.acc,
                               (size_t)2 * pqn * N, batch, s));
      if (no_fold && fuse && rs_out) {
        TRY(do_moddown_rescale(ctx, lv, w.acc, 2 * pqn, rs_out, 2 * lv, w.F, w.C, batch, s));
        return HELRM_OK;
      }
      if (!no_fold && fuse) {
        TRY(do_moddown_modup(ctx, lv, w.acc, 2 * pqn, zbuf, 2 * qn, w.F, f_bs, w.C, batch, s));
        z_digits = true;
      } else {
        TRY(do_moddown(ctx, lv, w.acc, 2 * pqn, no_fold ? out : zbuf, 2 * qn, w.mdP, w.mdT, batch, s));
      }
      z = zbuf;
    }
  }
  // 5. fold stages
  for (size_t si = 0; si < p->stages.size(); si++) {
    const int st = p->stages[si].first, r = p->stages[si].second;
    if (!z_digits) TRY(do_modup(ctx, lv, z + (size_t)qn * N, 2 * qn, D, f_bs, w.coef, batch, s));
    std::vector<KsTerm> terms;
    for (int t = 1; t < r; t++) {
      KsTerm k;
      k.digits = D;
      k.c0 = z;
      TRY(key_for(ctx, (long)t * st, &k));
      terms.push_back(k);
    }
    if ((int)terms.size() > HELRM_MAX_TERMS) {
      set_error("fold radix above %d is not supported", HELRM_MAX_TERMS + 1);
      return HELRM_EINVAL;
    }
    TRY(launch_ks_accumulate(ctx, lv, terms.data(), (int)terms.size(), (size_t)f_bs * N, (size_t)2 * qn * N,
                             z, (size_t)2 * qn * N, w.acc, (size_t)2 * pqn * N, batch, s));
    const bool last = si + 1 == p->stages.size();
    if (last && fuse && rs_out) {
      TRY(do_moddown_rescale(ctx, lv, w.acc, 2 * pqn, rs_out, 2 * lv, w.F, w.C, batch, s));
      return HELRM_OK;
    }
    u64 *dst = last ? out : (z == w.zA ? w.zB : w.zA);
    if (!last && fuse) {
      TRY(do_moddown_modup(ctx, lv, w.acc, 2 * pqn, dst, 2 * qn, w.F, f_bs, w.C, batch, s));
      z_digits = true;
    } else {
      TRY(do_moddown(ctx, lv, w.acc, 2 * pqn, dst, 2 * qn, w.mdP, w.mdT, batch, s));
      z_digits = false;
    }
    z = dst;
  }
  if (rs_out) TRY(do_rescale(ctx, lv, out, 2 * qn, rs_out, 2 * lv, w.top, w.V, batch, s));
  return HELRM_OK;
}

// ---------------------------------------------------------------- mixed batches

// A batch whose ciphertexts use different plans (uneven packings of the same
// level, baby-step count n1 and rotation direction; the giant-step counts may
// differ, and the per-element buffers are laid out for the largest).
// The elements are taken in plan groups; groups with more fold stages come
// first, so at every fold stage the elements still folding are a prefix of
// the batch.
struct PlanGroup {
  const helrm_plan *p;
  int start, count;
};

int mixed_groups(const helrm_ctx *c, const helrm_plan *const *plans, int batch, std::vector<PlanGroup> &groups,
                 std::vector<int> &order) {
  CHECK_ARG(plans && batch >= 1, "need one plan per batch element");
  const helrm_plan *p0 = plans[0];
  CHECK_ARG(p0 && p0->ctx == c, "NULL or foreign plan 0");
  std::vector<const helrm_plan *> uniq;
  for (int b = 0; b < batch; b++) {
    const helrm_plan *q = plans[b];
    CHECK_ARG(q && q->ctx == c, "NULL or foreign plan for element %d", b);
    CHECK_ARG(q->level == p0->level && q->n1 == p0->n1 && q->sign == p0->sign,
              "element %d: plans of one batch share level, n1 and rotation direction", b);
    const bool g0 = q->giants.size() == 1 && q->giants[0] == 0, f0 = p0->giants.size() == 1 && p0->giants[0] == 0;
    CHECK_ARG(g0 == f0, "element %d: either every plan or none has giant steps beyond g = 0", b);
    if (std::find(uniq.begin(), uniq.end(), q) == uniq.end()) uniq.push_back(q);
  }
  std::stable_sort(uniq.begin(), uniq.end(), [](const helrm_plan *a, const helrm_plan *b) {
    return a->stages.size() > b->stages.size();
  });
  groups.clear();
  order.clear();
  for (const helrm_plan *q : uniq) {
    PlanGroup g{q, (int)order.size(), 0};
    for (int b = 0; b < batch; b++)
      if (plans[b] == q) {
        order.push_back(b);
        g.count++;
      }
    groups.push_back(g);
  }
  return HELRM_OK;
}

// The plan of a mixed batch with the most giant steps: the workspace is carved for it.
const helrm_plan *widest(const std::vector<PlanGroup> &groups) {
  const helrm_plan *w = groups[0].p;
  for (auto &g : groups)
    if (g.p->n2 > w->n2) w = g.p;
  return w;
}

size_t mixed_ws_bytes(const helrm_ctx *c, const std::vector<PlanGroup> &groups, int batch) {
  std::vector<const helrm_plan *> ps;
  for (auto &g : groups) ps.push_back(g.p);
  const size_t ngu = nonzero_giants(ps.data(), (int)ps.size());
  const size_t N = c->N, lv = groups[0].p->level;
  return matvec_ws_bytes(c, widest(groups), batch, true, ngu) + rnd((size_t)batch * 2 * (lv + 1) * N) +
         rnd((size_t)batch * 2 * lv * N);
}

// The lookup of a mixed batch with the fused boundaries: the steps that do not
// depend on the plan (ModUp, the ModDown boundaries, the rescale) run once
// over the whole batch (or over the prefix still folding); the baby-step MAC
// and the key-switch accumulations run once per plan group.  ct: the sorted
// selectors ([batch][2][level+1]); rs_out: the sorted results ([batch][2][level]).
int run_mixed(helrm_ctx *ctx, const std::vector<PlanGroup> &groups, const u64 *ct, u64 *rs_out, int batch,
              MatvecWS &w, hipStream_t s) {
  const helrm_plan *p0 = groups[0].p;
  const int N = ctx->N, lv = p0->level, qn = lv + 1, pqn = lv + 1 + ctx->K, beta = ctx->n_digits(lv);
  const int n2 = widest(groups)->n2;   // X, xg and Dg hold n2 giants per element; plan g uses its first g.p->n2
  const size_t d_bs = (size_t)beta * pqn, f_bs = 2 * (size_t)qn + beta * pqn, ct_bs = 2 * (size_t)qn;
  const size_t x_bs = (size_t)n2 * 2 * pqn, c_bs = 2 * (size_t)pqn, rs_bs = 2 * (size_t)lv;
  u64 *const D = w.F + (size_t)2 * qn * N;
  const bool only0 = p0->giants.size() == 1 && p0->giants[0] == 0;
  // 1. hoisted ModUp of every c1
  TRY(do_modup(ctx, lv, ct + (size_t)qn * N, (int)ct_bs, D, (int)f_bs, w.coef, batch, s));
  // 2. fused baby steps + plaintext MAC, per plan group
  for (const PlanGroup &g : groups)
    for (int g0 = 0; g0 < g.p->n2; g0 += HELRM_MAX_GTILE) {
      const int ng = std::min(HELRM_MAX_GTILE, g.p->n2 - g0);
      TRY(launch_baby_mac(ctx, g.p, D + g.start * f_bs * N, f_bs * N, ct + g.start * ct_bs * N, ct_bs * N,
                          w.X + (g.start * x_bs + (size_t)g0 * 2 * pqn) * N, x_bs * N, g0, ng, g.count, s, false,
                          true, w.E ? w.E + g.start * fold_entry_words(ctx, lv) : nullptr));
    }
  // elements with no fold stage: the suffix of groups with stages == 0
  auto stages_of = [&](const PlanGroup &g) { return (int)g.p->stages.size(); };
  auto first_with_at_most = [&](int k) {   // first element whose plan has <= k stages
    for (const PlanGroup &g : groups)
      if (stages_of(g) <= k) return g.start;
    return batch;
  };
  const u64 *src = w.X;   // what the first boundary reads: X_0 (only g = 0) or the giant accumulators
  size_t src_bs = x_bs;
  if (!only0) {
    // 3. x_g = ModDown(X_g) for every giant of every element; 4. giant rotations
    TRY(do_moddown(ctx, lv, w.X, 2 * pqn, w.xg, 2 * qn, w.mdP, w.mdT, batch * n2, s));
    TRY(do_modup(ctx, lv, w.xg + (size_t)qn * N, 2 * qn, w.Dg, (int)d_bs, w.coef, batch * n2, s));
    for (const PlanGroup &g : groups) {
      std::vector<KsTerm> terms;
      bool has0 = false;
      for (int gi : g.p->giants) {
        if (gi == 0) {
          has0 = true;
          continue;
        }
        KsTerm t;
        t.digits = w.Dg + ((size_t)g.start * n2 + gi) * d_bs * N;
        t.c0 = w.xg + ((size_t)g.start * n2 + gi) * 2 * qn * N;
        TRY(key_for(ctx, (long)g.p->sign * g.p->n1 * gi, &t));
        terms.push_back(t);
      }
      TRY(launch_ks_accumulate(ctx, lv, terms.data(), (int)terms.size(), (size_t)n2 * d_bs * N,
                               (size_t)n2 * 2 * qn * N, has0 ? w.xg + (size_t)g.start * n2 * 2 * qn * N : nullptr,
                               (size_t)n2 * 2 * qn * N, w.acc + g.start * c_bs * N, c_bs * N, g.count, s));
    }
    src = w.acc;
    src_bs = c_bs;
  }
  // first boundary: ModDown -> rescale for the elements without fold stages,
  // ModDown -> ModUp (z in zA, its digits in F) for the others
  const int n_fold = first_with_at_most(0);
  if (n_fold < batch)
    TRY(do_moddown_rescale(ctx, lv, src + n_fold * src_bs * N, (int)src_bs, rs_out + n_fold * rs_bs * N,
                           (int)rs_bs, w.F + n_fold * f_bs * N, w.C + n_fold * c_bs * N, batch - n_fold, s));
  if (n_fold > 0)
    TRY(do_moddown_modup(ctx, lv, src, (int)src_bs, w.zA, 2 * qn, w.F, (int)f_bs, w.C, n_fold, s));
  // 5. fold stages: stage si runs for the prefix of elements with more than si stages
  u64 *z = w.zA, *zn = w.zB;
  const int max_st = stages_of(groups[0]);
  for (int si = 0; si < max_st; si++) {
    const int active = first_with_at_most(si);
    for (const PlanGroup &g : groups) {
      if (stages_of(g) <= si) break;
      const int st = g.p->stages[si].first, r = g.p->stages[si].second;
      std::vector<KsTerm> terms;
      for (int t = 1; t < r; t++) {
        KsTerm k;
        k.digits = D + g.start * f_bs * N;
        k.c0 = z + g.start * 2 * (size_t)qn * N;
        TRY(key_for(ctx, (long)t * st, &k));
        terms.push_back(k);
      }
      CHECK_ARG((int)terms.size() <= HELRM_MAX_TERMS, "fold radix above %d is not supported", HELRM_MAX_TERMS + 1);
      TRY(launch_ks_accumulate(ctx, lv, terms.data(), (int)terms.size(), f_bs * N, 2 * (size_t)qn * N,
                               z + g.start * 2 * (size_t)qn * N, 2 * (size_t)qn * N, w.acc + g.start * c_bs * N,
                               c_bs * N, g.count, s));
    }
    // elements whose last stage this is: [done0, active); the rest go on
    const int done0 = first_with_at_most(si + 1);
    if (done0 < active)
      TRY(do_moddown_rescale(ctx, lv, w.acc + done0 * c_bs * N, (int)c_bs, rs_out + done0 * rs_bs * N, (int)rs_bs,
                             w.F + done0 * f_bs * N, w.C + done0 * c_bs * N, active - done0, s));
    if (done0 > 0) {
      TRY(do_moddown_modup(ctx, lv, w.acc, (int)c_bs, zn, 2 * qn, w.F, (int)f_bs, w.C, done0, s));
      std::swap(z, zn);
    }
  }
  return HELRM_OK;
}

// Selectors into plan-group order (sel -> dst) or results back (src -> out),
// one copy per run of consecutive elements.
int permute_elements(const std::vector<int> &order, const u64 *from, u64 *to, size_t words, bool gather,
                     hipStream_t s) {
  const int n = (int)order.size();
  for (int i = 0; i < n;) {
    int j = i + 1;
    while (j < n && order[j] == order[j - 1] + 1) j++;
    const size_t src = gather ? (size_t)order[i] : (size_t)i, dst = gather ? (size_t)i : (size_t)order[i];
    HIP_TRY(hipMemcpyAsync(to + dst * words, from + src * words, (size_t)(j - i) * words * sizeof(u64),
                           hipMemcpyDeviceToDevice, s));
    i = j;
  }
  return HELRM_OK;
}

// Whole mixed-batch lookup on a workspace that mixed_ws_bytes sized.
int lookup_mixed(helrm_ctx *c, const std::vector<PlanGroup> &groups, const std::vector<int> &order,
                 const u64 *sel, int batch, u64 *out, char *base, hipStream_t s) {
  const helrm_plan *p0 = widest(groups);
  const size_t N = c->N, lv = p0->level, in_words = 2 * (lv + 1) * N, out_words = 2 * lv * N;
  const bool fuse = c->tune_fuse_ks && fused_fits(c, (int)lv);
  std::vector<const helrm_plan *> ps;
  for (auto &g : groups) ps.push_back(g.p);
  const size_t ngu = nonzero_giants(ps.data(), (int)ps.size());
  MatvecWS w = carve_matvec(c, p0, batch, true, base, ngu);
  bool ident = true;
  for (int i = 0; i < batch; i++) ident = ident && order[i] == i;
  u64 *s_sel = (u64 *)(base + matvec_ws_bytes(c, p0, batch, true, ngu));
  u64 *s_out = (u64 *)((char *)s_sel + rnd((size_t)batch * in_words / N * N));
  const u64 *in = sel;
  u64 *res = out;
  if (!ident) {
    TRY(permute_elements(order, sel, s_sel, in_words, true, s));
    in = s_sel;
    res = s_out;
  }
  if (fuse) {
    TRY(run_mixed(c, groups, in, res, batch, w, s));
  } else {
    // plain ModDown order: one lookup per plan group
    for (const PlanGroup &g : groups) {
      MatvecWS wg = carve_matvec(c, g.p, g.count, true, base);
      TRY(run_matvec(c, &g.p, 1, in + g.start * in_words, 2 * (int)(lv + 1), wg.mv, res + g.start * out_words,
                     g.count, wg, s));
    }
  }
  if (!ident) TRY(permute_elements(order, s_out, out, out_words, false, s));
  return HELRM_OK;
}

LimbList ll_from_primes(helrm_ctx *ctx, int n_limbs, const int32_t *prime_index, int off0) {
  LimbList ll = ll_make(n_limbs, n_limbs, n_limbs);
  for (int i = 0; i < n_limbs; i++) {
    ll.src_off[i] = off0 + i;
    ll.dst_off[i] = off0 + i;
    ll.prime[i] = (unsigned char)prime_index[i];
  }
  return ll;
}

int check_primes(const helrm_ctx *ctx, int n_limbs, const int32_t *prime_index) {
  CHECK_ARG(n_limbs >= 0, "n_limbs must be >= 0");
  CHECK_ARG(n_limbs == 0 || prime_index, "prime_index is NULL");
  for (int i = 0; i < n_limbs; i++)
    CHECK_ARG(prime_index[i] >= 0 && prime_index[i] < ctx->nprimes, "prime_index[%d] = %d out of range", i,
              prime_index[i]);
  return HELRM_OK;
}

}  // namespace

// ================================================================ C ABI

static int check_multi_plans(const helrm_ctx *c, const helrm_plan *const *plans, int n_in);

// Blocks of 2^lb consecutive coefficients in chain order.  Coefficient x is
// the evaluation at the exponent e = 2 brv(x) + 1 (mod 2N); the block of x
// is the class of e modulo 2N / 2^lb, so every Galois map sends a block onto
// a block, and the rotation by 5^b sends the class (-1)^s 5^i to (-1)^s
// 5^(i+b).  Position s n/2 + i of the chain (n = N / 2^lb blocks) holds the
// block of class (-1)^s 5^i.  Returns false unless that is a permutation.
static bool block_chain(int logn, int lb, std::vector<u64> &chain) {
  const int bits = logn - lb;                     // bits of a block index
  const u64 nblk = 1ull << bits, half = nblk / 2;
  const u64 mask = (2ull << bits) - 1;            // exponents modulo 2N / 2^lb
  chain.assign(nblk, 0);
  std::vector<char> seen(nblk, 0);
  u64 pw = 1;
  for (u64 i = 0; i < half; i++) {
    for (int sg = 0; sg < 2; sg++) {
      const u64 e = sg ? (0 - pw) & mask : pw;
      const u64 v = (e - 1) / 2;
      u64 m = 0;
      for (int k = 0; k < bits; k++) m |= ((v >> k) & 1) << (bits - 1 - k);
      if (m >= nblk || seen[m]) return false;
      seen[m] = 1;
      chain[sg * half + i] = m;
    }
    pw = (pw * 5) & mask;
  }
  return true;
}

extern "C" int helrm_create(const helrm_params *prm, helrm_ctx **out) {
  API_GUARD_BEGIN
  CHECK_ARG(prm && out, "NULL argument");
  *out = nullptr;
  CHECK_ARG(prm->log_n == 12 || prm->log_n == 16, "log_n must be 12 or 16");
  CHECK_ARG(prm->L >= 0 && prm->K >= 1 && prm->K <= 16 && prm->alpha >= 1 && prm->alpha <= 16,
            "bad L/K/alpha");
  CHECK_ARG(prm->L + 1 + prm->K <= HELRM_MAX_PRIMES, "too many primes");
  CHECK_ARG(prm->q && prm->p, "NULL prime arrays");
  helrm_ctx *c = new helrm_ctx();
  c->logn = prm->log_n;
  c->N = 1 << prm->log_n;
  c->L = prm->L;
  c->K = prm->K;
  c->alpha = prm->alpha;
  c->dnum = (prm->L + 1 + prm->alpha - 1) / prm->alpha;
  c->nprimes = prm->L + 1 + prm->K;
  for (int i = 0; i <= prm->L; i++) c->primes.push_back(prm->q[i]);
  for (int i = 0; i < prm->K; i++) c->primes.push_back(prm->p[i]);
  const u64 twoN = 2ull * c->N;
  for (int i = 0; i < c->nprimes; i++) {
    const u64 q = c->primes[i];
    if (q < 3 || q >= (1ull << 60) || q % twoN != 1) {
      set_error("prime %d (%llu) must be < 2^60 and = 1 mod 2N", i, (unsigned long long)q);
      delete c;
      return HELRM_EINVAL;
    }
    for (int k = 0; k < i; k++)
      if (c->primes[k] == q) {
        set_error("prime %d repeated", i);
        delete c;
        return HELRM_EINVAL;
      }
  }
  if (c->dnum > 16 || c->alpha > 16) {
    set_error("at most 16 digits of at most 16 primes");
    delete c;
    return HELRM_EINVAL;
  }
  int rc = hipGetDevice(&c->device);
  if (rc != hipSuccess) {
    set_error("hipGetDevice failed");
    delete c;
    return HELRM_EHIP;
  }
  // the current device is c->device here: resolve its static scratch once
  if (scratch_address(c->device, &c->noalloc_scratch) != HELRM_OK) {
    delete c;
    return HELRM_EHIP;
  }
  const int N = c->N;
  // roots: psi = x^((q-1)/2N) for the smallest non-residue x
  std::vector<TW> twf((size_t)c->nprimes * N), twi((size_t)c->nprimes * N);
  u64 P_all[HELRM_MAX_PRIMES];
  for (int i = 0; i < c->nprimes; i++) {
    const u64 q = c->primes[i];
    u64 x = 2;
    while (hpow(x, (q - 1) / 2, q) != q - 1) x++;
    const u64 psi = hpow(x, (q - 1) / twoN, q);
    c->psi.push_back(psi);
    const u64 psii = hinv(psi, q);
    std::vector<u64> pw(N), pwi(N);
    pw[0] = pwi[0] = 1;
    for (int k = 1; k < N; k++) { pw[k] = hmul(pw[k - 1], psi, q); pwi[k] = hmul(pwi[k - 1], psii, q); }
    for (int k = 0; k < N; k++) {
      const unsigned e = brv((unsigned)k, c->logn);
      twf[(size_t)i * N + k] = tw_of(pw[e], q);
      twi[(size_t)i * N + k] = tw_of(pwi[e], q);
    }
    u64 Pm = 1;
    for (int k = 0; k < c->K; k++) Pm = hmul(Pm, c->primes[c->L + 1 + k] % q, q);
    P_all[i] = Pm;
    PrimeInfo pi;
    pi.q = q;
    pi.qn = neg_inv64(q);
    pi.mu = (u64)(((u128)1 << 64) / q);
    const u64 r1 = (u64)(((u128)1 << 64) % q);
    pi.r2 = hmul(r1, r1, q);
    pi.ninv = hinv((u64)N % q, q);
    pi.ninv_p = shoup_of(pi.ninv, q);
    pi.pmod = Pm;
    pi.pmod_p = shoup_of(Pm, q);
    pi.pinv = Pm ? hinv(Pm, q) : 0;
    pi.pinv_p = shoup_of(pi.pinv, q);
    pi.qd = (double)q;
    pi.qinv_d = 1.0 / (double)q;
    pi.ninv_d = (double)pi.ninv;
    pi.lam = (u64)0 - (u64)(((u128)1 << 64) % q);
    c->h_pinfo.push_back(pi);
  }
  std::vector<double> twdf(twf.size()), twdi(twi.size());
  for (size_t k = 0; k < twf.size(); k++) {
    twdf[k] = (double)twf[k].w;
    twdi[k] = (double)twi[k].w;
  }
  // conversion tables
  ConstBuilder cb;
  struct Fix { int level, digit; size_t inv, mont; };
  std::vector<Fix> fix_up, fix_down;
  std::vector<size_t> off_pinv(c->L + 1), off_qinv(c->L + 1);
  c->modup_tabs.resize(c->L + 1);
  c->moddown_tabs.resize(c->L + 1);
  for (int lv = 0; lv <= c->L; lv++) {
    const int beta = c->n_digits(lv), pqn = lv + 1 + c->K;
    c->modup_tabs[lv].resize(beta);
    for (int j = 0; j < beta; j++) {
      std::vector<int> in, outp;
      for (int i = c->digit_lo(j); i < c->digit_hi(j, lv); i++) in.push_back(i);
      for (int r = 0; r < pqn; r++)
        if (r < c->digit_lo(j) || r >= c->digit_hi(j, lv)) outp.push_back(c->pq_prime(r, lv));
      Fix f{lv, j, 0, 0};
      build_conv(c, cb, in, outp, c->modup_tabs[lv][j], f.inv, f.mont);
      fix_up.push_back(f);
    }
    std::vector<int> in, outp;
    for (int k = 0; k < c->K; k++) in.push_back(c->L + 1 + k);
    for (int i = 0; i <= lv; i++) outp.push_back(i);
    Fix f{lv, 0, 0, 0};
    build_conv(c, cb, in, outp, c->moddown_tabs[lv], f.inv, f.mont);
    fix_down.push_back(f);
    std::vector<TW> pinv;
    for (int p = 0; p < 2; p++)
      for (int i = 0; i <= lv; i++) pinv.push_back(TW{c->h_pinfo[i].pinv, c->h_pinfo[i].pinv_p});
    off_pinv[lv] = cb.add_tw(pinv);
    std::vector<TW> qinv;
    for (int p = 0; p < 2; p++)
      for (int i = 0; i < lv; i++) qinv.push_back(tw_of(hinv(c->primes[lv] % c->primes[i], c->primes[i]), c->primes[i]));
    if (qinv.empty()) qinv.push_back(TW{0, 0});
    off_qinv[lv] = cb.add_tw(qinv);
  }
  // coefficient blocks in chain order (blocks of 8, 64 and 256)
  size_t off_chain[3];
  {
    const int lbs[3] = {3, 6, 8};
    for (int k = 0; k < 3; k++) {
      std::vector<u64> chain;
      if (!block_chain(c->logn, lbs[k], chain)) {
        set_error("internal: coefficient block chain is not a permutation");
        delete c;
        return HELRM_EINVAL;
      }
      off_chain[k] = cb.add_u64(chain);
    }
  }
  auto fail = [&](int code) {
    helrm_destroy(c);
    return code;
  };
  if (hipMalloc(&c->d_pinfo, sizeof(PrimeInfo) * c->nprimes) != hipSuccess ||
      hipMalloc(&c->d_tw_fwd, sizeof(TW) * twf.size()) != hipSuccess ||
      hipMalloc(&c->d_tw_inv, sizeof(TW) * twi.size()) != hipSuccess ||
      hipMalloc(&c->d_twd_fwd, sizeof(double) * twf.size()) != hipSuccess ||
      hipMalloc(&c->d_twd_inv, sizeof(double) * twi.size()) != hipSuccess ||
      hipMalloc(&c->d_const, sizeof(u64) * cb.words.size()) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of context tables failed");
    return fail(HELRM_ENOMEM);
  }
  if (hipMemcpy(c->d_pinfo, c->h_pinfo.data(), sizeof(PrimeInfo) * c->nprimes, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(c->d_tw_fwd, twf.data(), sizeof(TW) * twf.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_tw_inv, twi.data(), sizeof(TW) * twi.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_twd_fwd, twdf.data(), sizeof(double) * twdf.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_twd_inv, twdi.data(), sizeof(double) * twdi.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_const, cb.words.data(), sizeof(u64) * cb.words.size(), hipMemcpyHostToDevice) !=
          hipSuccess) {
    set_error("upload of context tables failed");
    return fail(HELRM_EHIP);
  }
  for (auto &f : fix_up) {
    c->modup_tabs[f.level][f.digit].hat_inv = (const TW *)(c->d_const + f.inv);
    c->modup_tabs[f.level][f.digit].hat_mont = c->d_const + f.mont;
  }
  for (auto &f : fix_down) {
    c->moddown_tabs[f.level].hat_inv = (const TW *)(c->d_const + f.inv);
    c->moddown_tabs[f.level].hat_mont = c->d_const + f.mont;
  }
  c->d_block_chain = c->d_const + off_chain[0];
  c->d_chain64 = c->d_const + off_chain[1];
  c->d_chain256 = c->d_const + off_chain[2];
  c->moddown_pinv.resize(c->L + 1);
  c->rescale_qinv.resize(c->L + 1);
  for (int lv = 0; lv <= c->L; lv++) {
    c->moddown_pinv[lv] = (const TW *)(c->d_const + off_pinv[lv]);
    c->rescale_qinv[lv] = (const TW *)(c->d_const + off_qinv[lv]);
  }
  *out = c;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_destroy(helrm_ctx *c) {
  API_GUARD_BEGIN
  if (!c) return HELRM_OK;
  (void)hipDeviceSynchronize();
  timing_clear(c);
  for (auto e : c->evpool) (void)hipEventDestroy(e);
  for (auto &kv : c->keys) (void)hipFree(kv.second.d);
  for (auto &kv : c->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  for (void *p : c->ws_retired) (void)hipFree(p);
  if (c->d_pinfo) (void)hipFree(c->d_pinfo);
  if (c->d_tw_fwd) (void)hipFree(c->d_tw_fwd);
  if (c->d_tw_inv) (void)hipFree(c->d_tw_inv);
  if (c->d_twd_fwd) (void)hipFree(c->d_twd_fwd);
  if (c->d_twd_inv) (void)hipFree(c->d_twd_inv);
  if (c->d_const) (void)hipFree(c->d_const);
  delete c;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_get_psi(const helrm_ctx *c, int i, uint64_t *psi) {
  CHECK_ARG(c && psi, "NULL argument");
  CHECK_ARG(i >= 0 && i < c->nprimes, "prime index out of range");
  *psi = c->psi[i];
  return HELRM_OK;
}

extern "C" int helrm_load_eval_keys(helrm_ctx *c, const uint32_t *galois, int n_keys, const uint64_t *keys,
                                    const uint64_t *seeds) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(n_keys >= 0, "n_keys < 0");
  CHECK_ARG(n_keys == 0 || (galois && keys), "NULL galois or keys");
  const size_t N = c->N, kl = c->L + 1 + c->K;
  const size_t words = key_words(c->dnum, (int)kl, (int)N);
  const size_t bytes = key_bytes(c->dnum, (int)kl, (int)N);
  for (int k = 0; k < n_keys; k++)
    CHECK_ARG(galois[k] == 0 || (galois[k] & 1u) && galois[k] < 2u * c->N, "bad galois element %u", galois[k]);
  for (int k = 0; k < n_keys; k++) {
    u64 *d = nullptr;
    auto it = c->keys.find(galois[k]);
    if (it != c->keys.end()) {
      d = it->second.d;
    } else {
      if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("key allocation (%zu bytes) failed", bytes);
        return HELRM_ENOMEM;
      }
      c->keys[galois[k]] = KeyEntry{d};
    }
    c->keys[galois[k]].seed = seeds ? seeds[k] : 0;
    c->keys[galois[k]].seeded = seeds != nullptr;
    HIP_TRY(hipMemcpy(d, keys + (size_t)k * words, words * sizeof(u64), hipMemcpyDefault));
    LimbList ll = ll_make((int)kl, (int)kl, (int)kl);
    for (size_t i = 0; i < kl; i++) { ll.src_off[i] = (int)i; ll.dst_off[i] = (int)i; ll.prime[i] = (unsigned char)i; }
    TRY(launch_to_mont(c, d, ll, c->dnum * 2, 0));
    TRY(launch_pack_key(c, d, 0));
  }
  if (n_keys > 0) c->keys_gen++;   // folded plan operands built from earlier keys are stale now
  HIP_TRY(hipDeviceSynchronize());
  return HELRM_OK;
  API_GUARD_END
}

static int ntt_common(helrm_ctx *c, uint64_t *d, int n_limbs, const int32_t *pidx, int batch, void *stream,
                      bool fwd) {
  CHECK_ARG(c && (d || n_limbs * batch == 0), "NULL argument");
  CHECK_ARG(batch >= 0, "batch < 0");
  TRY(check_primes(c, n_limbs, pidx));
  for (int i0 = 0; i0 < n_limbs; i0 += HELRM_MAX_LIMBS) {
    const int n = std::min(HELRM_MAX_LIMBS, n_limbs - i0);
    LimbList ll = ll_from_primes(c, n, pidx + i0, i0);
    ll.src_bstride = ll.dst_bstride = n_limbs;
    TRY(launch_ntt(c, d, d, ll, batch, fwd, as_stream(stream)));
  }
  return HELRM_OK;
}

extern "C" int helrm_ntt(helrm_ctx *c, uint64_t *d, int n_limbs, const int32_t *pidx, int batch, void *stream) {
  API_GUARD_BEGIN
  return ntt_common(c, d, n_limbs, pidx, batch, stream, true);
  API_GUARD_END
}

extern "C" int helrm_intt(helrm_ctx *c, uint64_t *d, int n_limbs, const int32_t *pidx, int batch, void *stream) {
  API_GUARD_BEGIN
  return ntt_common(c, d, n_limbs, pidx, batch, stream, false);
  API_GUARD_END
}

extern "C" int helrm_automorph(helrm_ctx *c, const uint64_t *in, uint64_t *out, uint32_t galois, int n_limbs,
                               int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(n_limbs >= 0 && batch >= 0, "negative size");
  CHECK_ARG(n_limbs * batch == 0 || (in && out), "NULL buffer");
  CHECK_ARG((galois & 1u) && galois < 2u * c->N, "galois element must be odd and < 2N");
  CHECK_ARG(n_limbs * batch == 0 || in != out, "in and out must differ");
  return launch_automorph(c, in, out, galois, n_limbs, batch, as_stream(stream));
  API_GUARD_END
}

extern "C" int helrm_poly_op(helrm_ctx *c, int op, const uint64_t *a, const uint64_t *b, uint64_t *out,
                             int n_limbs, const int32_t *pidx, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(op >= 0 && op <= 3, "bad op");
  CHECK_ARG(batch >= 0, "batch < 0");
  TRY(check_primes(c, n_limbs, pidx));
  CHECK_ARG(n_limbs * batch == 0 || (a && out && (op == HELRM_OP_NEG || b)), "NULL buffer");
  for (int i0 = 0; i0 < n_limbs; i0 += HELRM_MAX_LIMBS) {
    const int n = std::min(HELRM_MAX_LIMBS, n_limbs - i0);
    LimbList ll = ll_from_primes(c, n, pidx + i0, i0);
    ll.src_bstride = ll.dst_bstride = n_limbs;
    TRY(launch_poly_op(c, op, a, b ? b : a, out, ll, batch, as_stream(stream)));
  }
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_mul_scalar(helrm_ctx *c, const uint64_t *a, const uint64_t *scalars, uint64_t *out,
                                int n_limbs, const int32_t *pidx, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(batch >= 0, "batch < 0");
  TRY(check_primes(c, n_limbs, pidx));
  CHECK_ARG(n_limbs * batch == 0 || (a && out && scalars), "NULL buffer");
  if (n_limbs * batch == 0) return HELRM_OK;   // before the scalars are read: they may be NULL
  for (int i0 = 0; i0 < n_limbs; i0 += 64) {
    const int n = std::min(64, n_limbs - i0);
    LimbList ll = ll_from_primes(c, n, pidx + i0, i0);
    ll.src_bstride = ll.dst_bstride = n_limbs;
    TRY(launch_mul_scalar(c, a, scalars + i0, out, ll, batch, as_stream(stream)));
  }
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_from_signed(helrm_ctx *c, const int64_t *in, uint64_t *out, int n_limbs,
                                 const int32_t *pidx, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(batch >= 0, "batch < 0");
  TRY(check_primes(c, n_limbs, pidx));
  CHECK_ARG(n_limbs * batch == 0 || (in && out), "NULL buffer");
  for (int i0 = 0; i0 < n_limbs; i0 += HELRM_MAX_LIMBS) {
    const int n = std::min(HELRM_MAX_LIMBS, n_limbs - i0);
    LimbList ll = ll_from_primes(c, n, pidx + i0, i0);
    ll.dst_bstride = n_limbs;
    TRY(launch_from_signed(c, in, out, ll, batch, as_stream(stream)));
  }
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_keyswitch_hoisted(helrm_ctx *c, const uint64_t *ct, int level, const int32_t *steps,
                                       int n_rot, uint64_t *out, int out_basis, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(level >= 0 && level <= c->L, "level %d out of range", level);
  CHECK_ARG(n_rot >= 0 && batch >= 0, "negative size");
  CHECK_ARG(out_basis == HELRM_BASIS_Q || out_basis == HELRM_BASIS_PQ, "bad out_basis");
  if (n_rot == 0 || batch == 0) return HELRM_OK;
  CHECK_ARG(ct && out && steps, "NULL buffer");
  hipStream_t s = as_stream(stream);
  const size_t N = c->N;
  const int qn = level + 1, pqn = level + 1 + c->K, beta = c->n_digits(level);
  std::vector<KsTerm> terms(n_rot);
  for (int r = 0; r < n_rot; r++) {
    terms[r].digits = nullptr;
    terms[r].c0 = ct;
    if (steps[r] % (c->N / 2) != 0) TRY(key_for(c, steps[r], &terms[r]));
    else terms[r].galois = 1;
  }
  KsSizes z = ks_sizes(c, level, batch, 1);
  size_t bytes = rnd(z.coef) + rnd(z.D) + rnd(z.X) + rnd(z.mdP) + rnd(z.mdT);
  char *base;
  TRY(ensure_ws(c, s, bytes, &base));
  Arena a{base};
  u64 *coef = a.take(z.coef), *D = a.take(z.D), *X = a.take(z.X), *mdP = a.take(z.mdP), *mdT = a.take(z.mdT);
  const int ct_bs = 2 * qn, d_bs = beta * pqn;
  TRY(do_modup(c, level, ct + (size_t)qn * N, ct_bs, D, d_bs, coef, batch, s));
  const int ob = out_basis == HELRM_BASIS_PQ ? 2 * pqn : 2 * qn;
  for (int r = 0; r < n_rot; r++) {
    u64 *dst = out + (size_t)r * ob * N;
    const size_t out_bs = (size_t)n_rot * ob * N;
    if (terms[r].galois == 1) {
      if (out_basis == HELRM_BASIS_PQ) {
        TRY(launch_ks_accumulate(c, level, nullptr, 0, 0, 0, ct, (size_t)ct_bs * N, dst, out_bs, batch, s));
      } else {
        LimbList cp = ll_make(2 * qn, ct_bs, n_rot * ob);
        for (int i = 0; i < 2 * qn; i++) { cp.src_off[i] = i; cp.dst_off[i] = i; cp.prime[i] = 0; }
        TRY(launch_copy_limbs(ct, dst, cp, batch, (int)N, s));
      }
      continue;
    }
    KsTerm t = terms[r];
    t.digits = D;
    if (out_basis == HELRM_BASIS_PQ) {
      TRY(launch_ks_accumulate(c, level, &t, 1, (size_t)d_bs * N, (size_t)ct_bs * N, nullptr, 0, dst, out_bs,
                               batch, s));
    } else {
      TRY(launch_ks_accumulate(c, level, &t, 1, (size_t)d_bs * N, (size_t)ct_bs * N, nullptr, 0, X,
                               (size_t)2 * pqn * N, batch, s));
      TRY(do_moddown(c, level, X, 2 * pqn, dst, n_rot * ob, mdP, mdT, batch, s));
    }
  }
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_rescale(helrm_ctx *c, const uint64_t *in, int level, uint64_t *out, int batch,
                             void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(level >= 1 && level <= c->L, "level %d out of range (1..L)", level);
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(in && out, "NULL buffer");
  hipStream_t s = as_stream(stream);
  const size_t N = c->N;
  size_t bytes = rnd((size_t)batch * 2 * N) + rnd((size_t)batch * 2 * level * N);
  char *base;
  TRY(ensure_ws(c, s, bytes, &base));
  Arena a{base};
  u64 *top = a.take((size_t)batch * 2 * N), *V = a.take((size_t)batch * 2 * level * N);
  return do_rescale(c, level, in, 2 * (level + 1), out, 2 * level, top, V, batch, s);
  API_GUARD_END
}

extern "C" int helrm_key_uniform(helrm_ctx *c, uint64_t seed, int digit, uint64_t *out, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && out, "NULL argument");
  CHECK_ARG(digit >= 0 && digit < c->dnum, "digit %d out of range", digit);
  return launch_key_uniform(c, seed, digit, out, as_stream(stream));
  API_GUARD_END
}

extern "C" int helrm_mul_relin(helrm_ctx *c, const uint64_t *a, const uint64_t *b, int level, uint64_t *out,
                               int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(level >= 0 && level <= c->L, "level %d out of range", level);
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(a && b && out, "NULL buffer");
  auto it = c->keys.find(0u);
  CHECK_ARG(it != c->keys.end(), "no relinearisation key loaded (galois element 0)");
  hipStream_t s = as_stream(stream);
  const size_t N = c->N;
  const int qn = level + 1, pqn = level + 1 + c->K, beta = c->n_digits(level);
  KsSizes z = ks_sizes(c, level, batch, 1);
  const size_t dw = (size_t)batch * 3 * qn * N;
  size_t bytes = rnd(dw) + rnd(z.coef) + rnd(z.D) + rnd(z.X) + rnd(z.mdP) + rnd(z.mdT);
  char *base;
  TRY(ensure_ws(c, s, bytes, &base));
  Arena ar{base};
  u64 *d = ar.take(dw), *coef = ar.take(z.coef), *D = ar.take(z.D), *X = ar.take(z.X), *mdP = ar.take(z.mdP),
      *mdT = ar.take(z.mdT);
  // 1. tensor product (d0, d1, d2)
  TRY(launch_tensor(c, a, b, d, level, batch, s));
  // 2. ModUp of d2, 3. key inner product with the relinearisation key plus
  //    P (d0, d1), 4. ModDown (P (d0, d1) passes through it as (d0, d1))
  const int d_bs = beta * pqn;
  TRY(do_modup(c, level, d + (size_t)2 * qn * N, 3 * qn, D, d_bs, coef, batch, s));
  KsTerm t;
  t.digits = D;
  t.c0 = nullptr;
  t.key = it->second.d;
  t.galois = 1;
  t.seed = it->second.seed;
  t.seeded = it->second.seeded;
  TRY(launch_ks_accumulate(c, level, &t, 1, (size_t)d_bs * N, 0, d, (size_t)3 * qn * N, X, (size_t)2 * pqn * N,
                           batch, s));
  TRY(do_moddown(c, level, X, 2 * pqn, out, 2 * qn, mdP, mdT, batch, s));
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_add_plain(helrm_ctx *c, const uint64_t *ct, const uint64_t *pt, int level, uint64_t *out,
                               int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(level >= 0 && level <= c->L, "level %d out of range", level);
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(ct && pt && out, "NULL buffer");
  return launch_add_plain(c, ct, pt, out, level, batch, as_stream(stream));
  API_GUARD_END
}

extern "C" int helrm_mod_drop(helrm_ctx *c, const uint64_t *in, int level_in, uint64_t *out, int level_out,
                              int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(level_in >= 0 && level_in <= c->L, "level_in %d out of range", level_in);
  CHECK_ARG(level_out >= 0 && level_out <= level_in, "level_out must be in [0, level_in]");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(in && out, "NULL buffer");
  CHECK_ARG(in != out, "in and out must differ");
  const int qi = level_in + 1, qo = level_out + 1;
  LimbList cp = ll_make(2 * qo, 2 * qi, 2 * qo);
  for (int cc = 0; cc < 2; cc++)
    for (int r = 0; r < qo; r++) {
      cp.src_off[cc * qo + r] = cc * qi + r;
      cp.dst_off[cc * qo + r] = cc * qo + r;
      cp.prime[cc * qo + r] = (unsigned char)r;
    }
  return launch_copy_limbs(in, out, cp, batch, c->N, as_stream(stream));
  API_GUARD_END
}

extern "C" int helrm_plan_create(helrm_ctx *c, const helrm_plan_desc *d, helrm_plan **out) {
  API_GUARD_BEGIN
  CHECK_ARG(c && d && out, "NULL argument");
  *out = nullptr;
  const int n = c->N / 2;
  CHECK_ARG(d->level >= 0 && d->level <= c->L, "plan level out of range");
  CHECK_ARG(is_pow2(d->m) && d->m <= n, "m must be a power of two <= N/2");
  CHECK_ARG(d->n1 >= 1 && d->n2 >= 1 && (long)d->n1 * d->n2 >= d->m, "need n1*n2 >= m");
  CHECK_ARG(d->n1 <= HELRM_MAX_BABY, "n1 above %d", HELRM_MAX_BABY);
  CHECK_ARG(d->radix >= 2 && d->radix <= HELRM_MAX_TERMS + 1, "radix must be in [2, %d]", HELRM_MAX_TERMS + 1);
  CHECK_ARG(d->n_diag >= 1 && d->diag && d->coeffs, "plan needs at least one diagonal");
  CHECK_ARG(d->sign == 1 || d->sign == -1, "sign must be +1 or -1");
  const int span = d->fold_span == 0 ? n : d->fold_span;
  CHECK_ARG(is_pow2(span) && span >= d->m && span <= n, "fold_span must be a power of two in [m, N/2]");
  for (int i = 0; i < d->n_diag; i++) {
    CHECK_ARG(d->diag[i] >= 0 && d->diag[i] < d->m, "diagonal index %d out of range", d->diag[i]);
    CHECK_ARG(i == 0 || d->diag[i] > d->diag[i - 1], "diagonal indices must ascend");
  }
  helrm_plan *p = new helrm_plan();
  p->ctx = c;
  p->level = d->level;
  p->m = d->m;
  p->n1 = d->n1;
  p->n2 = d->n2;
  p->radix = d->radix;
  p->n_diag = d->n_diag;
  p->sign = d->sign;
  p->span = span;
  p->slot.assign((size_t)d->n2 * d->n1, -1);
  for (int i = 0; i < d->n_diag; i++) {
    const int k = d->diag[i], g = k / d->n1, b = k % d->n1;
    p->diag.push_back(k);
    p->slot[(size_t)g * d->n1 + b] = i;
    if (std::find(p->babies.begin(), p->babies.end(), b) == p->babies.end()) p->babies.push_back(b);
    if (std::find(p->giants.begin(), p->giants.end(), g) == p->giants.end()) p->giants.push_back(g);
  }
  std::sort(p->babies.begin(), p->babies.end());
  std::sort(p->giants.begin(), p->giants.end());
  for (int sp = span; sp > d->m;) {
    const int r = std::min(d->radix, sp / d->m);
    const int st = sp / r;
    p->stages.push_back({st, r});
    sp = st;
  }
  const int pqn = d->level + 1 + c->K;
  p->pt_limb_stride = pqn;
  const size_t N = c->N;
  int64_t *dcoef = nullptr;
  auto fail = [&](int code) {
    if (dcoef) (void)hipFree(dcoef);
    helrm_plan_destroy(p);
    return code;
  };
  p->pt_words = (size_t)d->n_diag * pqn * N;
  if (hipMalloc(&p->d_pt, pt_bytes(p->pt_words)) != hipSuccess ||
      hipMalloc(&p->d_slot, p->slot.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&dcoef, (size_t)d->n_diag * N * sizeof(int64_t)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("plan allocation failed");
    return fail(HELRM_ENOMEM);
  }
  if (hipMemcpy(p->d_slot, p->slot.data(), p->slot.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dcoef, d->coeffs, (size_t)d->n_diag * N * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("plan upload failed");
    return fail(HELRM_EHIP);
  }
  LimbList ll = ll_make(pqn, pqn, pqn);
  for (int r = 0; r < pqn; r++) { ll.src_off[r] = r; ll.dst_off[r] = r; ll.prime[r] = (unsigned char)c->pq_prime(r, d->level); }
  int rc;
  if ((rc = launch_from_signed(c, dcoef, p->d_pt, ll, d->n_diag, 0)) != HELRM_OK) return fail(rc);
  if ((rc = launch_ntt(c, p->d_pt, p->d_pt, ll, d->n_diag, true, 0)) != HELRM_OK) return fail(rc);
  if ((rc = launch_to_mont(c, p->d_pt, ll, d->n_diag, 0)) != HELRM_OK) return fail(rc);
  if ((rc = launch_pack_pt(p->d_pt, p->pt_words, 0)) != HELRM_OK) return fail(rc);
  // matrix-core operands for batched launches of plans with several giant
  // steps: per giant tile of 8, the baby steps of the tile in the order the
  // baby-step launch takes them (ascending, b = 0 first).  Plans with fewer
  // baby steps than the matrix-core MAC's floor (mfma_min_slots, read here)
  // would never use them and keep none
  if (c->tune_ptm && d->n2 >= 2 && (int)p->babies.size() >= c->tune_mfma_min_slots) {
    const int tiles = (d->n2 + HELRM_MAX_GTILE - 1) / HELRM_MAX_GTILE;
    std::vector<int> tab((size_t)tiles * 64 * 8, -1);
    bool fits = true;
    for (int T = 0; T < tiles; T++) {
      int k = 0;
      for (int b : p->babies) {
        bool any = false;
        for (int g = 0; g < 8; g++) {
          const int G = T * 8 + g;
          if (G < d->n2 && p->slot[(size_t)G * d->n1 + b] >= 0) any = true;
        }
        if (!any) continue;
        if (k >= 64) { fits = false; break; }
        for (int g = 0; g < 8; g++) {
          const int G = T * 8 + g;
          tab[((size_t)T * 64 + k) * 8 + g] = G < d->n2 ? p->slot[(size_t)G * d->n1 + b] : -1;
        }
        k++;
      }
    }
    if (fits) {
      int *dtab = nullptr;
      const size_t bytes = (size_t)tiles * pqn * N * 4096;
      if (hipMalloc(&p->d_ptm, bytes) != hipSuccess || hipMalloc(&dtab, tab.size() * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        if (dtab) (void)hipFree(dtab);
        set_error("plan allocation failed (matrix-core operands)");
        return fail(HELRM_ENOMEM);
      }
      p->ptm_tiles = tiles;
      rc = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess
               ? launch_ptm_pack(c, p, dtab, 0)
               : HELRM_EHIP;
      if (rc == HELRM_OK && hipDeviceSynchronize() != hipSuccess) rc = HELRM_EHIP;
      (void)hipFree(dtab);
      if (rc != HELRM_OK) {
        set_error("plan preparation failed (matrix-core operands)");
        return fail(rc);
      }
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("plan preparation failed on the device");
    return fail(HELRM_EHIP);
  }
  (void)hipFree(dcoef);
  dcoef = nullptr;
  *out = p;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_plan_destroy(helrm_plan *p) {
  API_GUARD_BEGIN
  if (!p) return HELRM_OK;
  (void)hipDeviceSynchronize();
  if (p->d_pt) (void)hipFree(p->d_pt);
  if (p->d_slot) (void)hipFree(p->d_slot);
  if (p->d_ptm) (void)hipFree(p->d_ptm);
  if (p->d_wm) (void)hipFree(p->d_wm);
  delete p;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_plan_fold_keys(helrm_ctx *c, helrm_plan *p, size_t *bytes) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && p->ctx == c, "NULL or foreign plan");
  CHECK_ARG(c->n_digits(p->level) <= 3, "key folding supports at most 3 key-switching digits (level %d has %d)",
            p->level, c->n_digits(p->level));
  const int pqn = p->level + 1 + c->K, n1 = p->n1;
  const int tiles = (p->n2 + HELRM_MAX_GTILE - 1) / HELRM_MAX_GTILE;
  // depth: 4 entries per baby step of the tile, chunks of 64
  int kc = 1;
  for (int T = 0; T < tiles; T++) {
    int ns = 0;
    for (int b : p->babies) {
      bool any = false;
      for (int g = 0; g < HELRM_MAX_GTILE && T * HELRM_MAX_GTILE + g < p->n2; g++)
        if (p->slot[(size_t)(T * HELRM_MAX_GTILE + g) * n1 + b] >= 0) any = true;
      ns += any ? 1 : 0;
    }
    CHECK_ARG(ns <= HELRM_MAX_BABY, "key folding: at most %d baby steps per giant tile", HELRM_MAX_BABY);
    kc = std::max(kc, (4 * ns + 63) / 64);
  }
  std::vector<int> planes(pqn), off(pqn);
  int tot = 0;
  for (int r = 0; r < pqn; r++) {
    planes[r] = c->primes[c->pq_prime(r, p->level)] < SPLIT_MAC_LIMIT ? 5 : 8;
    off[r] = tot;
    tot += planes[r];
  }
  const size_t tile_bytes = (size_t)tot * c->N * kc * 1024;
  if (p->d_wm) {
    HIP_TRY(hipDeviceSynchronize());
    (void)hipFree(p->d_wm);
    p->d_wm = nullptr;
  }
  if (hipMalloc(&p->d_wm, tile_bytes * tiles) != hipSuccess) {
    (void)hipGetLastError();
    p->d_wm = nullptr;
    set_error("folded operands: allocation of %zu bytes failed", tile_bytes * tiles);
    return HELRM_ENOMEM;
  }
  p->wm_kc = kc;
  p->wm_tiles = tiles;
  p->wm_tile_bytes = tile_bytes;
  p->wm_planes = planes;
  p->wm_off = off;
  for (int T = 0; T < tiles; T++) {
    const int rc = launch_wfold_pack(c, p, T, 0);
    if (rc != HELRM_OK) {
      (void)hipFree(p->d_wm);
      p->d_wm = nullptr;
      return rc;
    }
  }
  HIP_TRY(hipDeviceSynchronize());
  p->wm_keys_gen = c->keys_gen;
  if (bytes) *bytes = tile_bytes * tiles;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_plan_rotation_steps(const helrm_plan *p, int32_t *steps, int cap, int *n) {
  API_GUARD_BEGIN
  CHECK_ARG(p && n, "NULL argument");
  std::vector<int> st;
  for (int b : p->babies)
    if (b) st.push_back(p->sign * b);
  for (int g : p->giants)
    if (g) st.push_back(p->sign * p->n1 * g);
  for (auto &sr : p->stages)
    for (int t = 1; t < sr.second; t++) st.push_back(t * sr.first);
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  *n = (int)st.size();
  for (int i = 0; i < (int)st.size() && i < cap; i++) steps[i] = st[i];
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_ptxt_ct_matvec_diag(helrm_ctx *c, const helrm_plan *p, const uint64_t *ct, uint64_t *out,
                                         int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && p->ctx == c, "NULL or foreign plan");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(ct && out, "NULL buffer");
  hipStream_t s = as_stream(stream);
  char *base;
  TRY(ensure_ws(c, s, matvec_ws_bytes(c, p, batch, false), &base));
  MatvecWS w = carve_matvec(c, p, batch, false, base);
  return run_matvec(c, &p, 1, ct, 2 * (p->level + 1), out, nullptr, batch, w, s);
  API_GUARD_END
}

extern "C" int helrm_lookup_packed(helrm_ctx *c, const helrm_plan *p, const uint64_t *sel, int batch,
                                   uint64_t *out, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && p->ctx == c, "NULL or foreign plan");
  CHECK_ARG(p->level >= 1, "lookup needs a plan at level >= 1");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(sel && out, "NULL buffer");
  hipStream_t s = as_stream(stream);
  char *base;
  TRY(ensure_ws(c, s, matvec_ws_bytes(c, p, batch, true), &base));
  MatvecWS w = carve_matvec(c, p, batch, true, base);
  return run_matvec(c, &p, 1, sel, 2 * (p->level + 1), w.mv, out, batch, w, s);
  API_GUARD_END
}

extern "C" int helrm_lookup_packed_noalloc(helrm_ctx *c, const helrm_plan *p, const uint64_t *sel, int batch,
                                           uint64_t *out, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && p->ctx == c, "NULL or foreign plan");
  CHECK_ARG(p->level >= 1, "lookup needs a plan at level >= 1");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(sel && out, "NULL buffer");
  CHECK_ARG(!c->timing, "kernel timing is enabled (it creates events): disable it for the no-allocation call");
  CHECK_ARG(c->noalloc_scratch, "the context has no static scratch");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  CHECK_ARG(dev == c->device, "the current device (%d) is not the context's (%d)", dev, c->device);
  const size_t bytes = matvec_ws_bytes(c, p, batch, true);
  if (bytes > (size_t)HELRM_NOALLOC_MAX_BYTES) {
    set_error("this lookup needs %zu bytes of scratch (level %d, batch %d); the static scratch holds %zu: use "
              "helrm_lookup_packed, or a smaller batch or level", bytes, p->level, batch,
              (size_t)HELRM_NOALLOC_MAX_BYTES);
    return HELRM_EINVAL;
  }
  MatvecWS w = carve_matvec(c, p, batch, true, c->noalloc_scratch);
  return run_matvec(c, &p, 1, sel, 2 * (p->level + 1), w.mv, out, batch, w, as_stream(stream));
  API_GUARD_END
}

extern "C" int helrm_lookup_multi(helrm_ctx *c, const helrm_plan *const *plans, int n_in, const uint64_t *sel,
                                  int batch, uint64_t *out, void *stream) {
  API_GUARD_BEGIN
  TRY(check_multi_plans(c, plans, n_in));
  const helrm_plan *p = plans[0];
  CHECK_ARG(p->level >= 1, "lookup needs plans at level >= 1");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(sel && out, "NULL buffer");
  hipStream_t s = as_stream(stream);
  const size_t ngu = nonzero_giants(plans, n_in);
  char *base;
  TRY(ensure_ws(c, s, matvec_ws_bytes(c, p, batch, true, ngu), &base));
  MatvecWS w = carve_matvec(c, p, batch, true, base, ngu);
  const int lv = p->level;
  return run_matvec(c, plans, n_in, sel, n_in * 2 * (lv + 1), w.mv, out, batch, w, s);
  API_GUARD_END
}

extern "C" int helrm_lookup_batch(helrm_ctx *c, const helrm_plan *const *plans, const uint64_t *sel, int batch,
                                  uint64_t *out, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(batch >= 0, "batch < 0");
  if (batch == 0) return HELRM_OK;
  CHECK_ARG(sel && out, "NULL buffer");
  std::vector<PlanGroup> groups;
  std::vector<int> order;
  TRY(mixed_groups(c, plans, batch, groups, order));
  CHECK_ARG(groups[0].p->level >= 1, "lookup needs plans at level >= 1");
  hipStream_t s = as_stream(stream);
  char *base;
  TRY(ensure_ws(c, s, mixed_ws_bytes(c, groups, batch), &base));
  return lookup_mixed(c, groups, order, sel, batch, out, base, s);
  API_GUARD_END
}

extern "C" int helrm_footprint_batch(const helrm_ctx *c, const helrm_plan *const *plans, int batch, size_t *bytes) {
  API_GUARD_BEGIN
  CHECK_ARG(c && bytes && batch >= 1, "bad argument");
  std::vector<PlanGroup> groups;
  std::vector<int> order;
  TRY(mixed_groups(c, plans, batch, groups, order));
  *bytes = mixed_ws_bytes(c, groups, batch);
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_reserve_batch(helrm_ctx *c, const helrm_plan *const *plans, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && batch >= 1, "bad argument");
  std::vector<PlanGroup> groups;
  std::vector<int> order;
  TRY(mixed_groups(c, plans, batch, groups, order));
  char *base;
  return ensure_ws(c, as_stream(stream), mixed_ws_bytes(c, groups, batch), &base);
  API_GUARD_END
}

extern "C" int helrm_footprint(const helrm_ctx *c, const helrm_plan *p, int batch, size_t *bytes) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && bytes && batch >= 0, "bad argument");
  *bytes = matvec_ws_bytes(c, p, batch, true);
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_reserve(helrm_ctx *c, const helrm_plan *p, int batch, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c && p && batch >= 0, "bad argument");
  char *base;
  return ensure_ws(c, as_stream(stream), matvec_ws_bytes(c, p, batch, true), &base);
  API_GUARD_END
}

extern "C" int helrm_release_stream(helrm_ctx *c, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  const hipStream_t s = as_stream(stream);
  std::lock_guard<std::mutex> lk(c->ws_mu);
  auto it = c->ws.find(s);
  if (it == c->ws.end()) return HELRM_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    cs = hipStreamCaptureStatusNone;
  }
  if (cs != hipStreamCaptureStatusNone) {
    set_error("the stream is being captured: its workspace cannot be released");
    return HELRM_ESTATE;
  }
  Workspace &w = it->second;
  if (w.ptr) {
    if (w.captured) {
      c->ws_retired.push_back(w.ptr);   // a captured graph may still use it
    } else {
      HIP_TRY(hipStreamSynchronize(s));
      void *p = w.ptr;
      c->ws.erase(it);   // forgotten before the free, so a failed free is never repeated
      HIP_TRY(hipFree(p));
      return HELRM_OK;
    }
  }
  c->ws.erase(it);
  return HELRM_OK;
  API_GUARD_END
}

// Plans of one multi-ciphertext lookup: same context, level, m, n1, n2,
// direction, fold radix and span.
static int check_multi_plans(const helrm_ctx *c, const helrm_plan *const *plans, int n_in) {
  CHECK_ARG(c && plans && n_in >= 1, "need at least one plan");
  const helrm_plan *p = plans[0];
  for (int i = 0; i < n_in; i++) {
    const helrm_plan *q = plans[i];
    CHECK_ARG(q && q->ctx == c, "NULL or foreign plan %d", i);
    CHECK_ARG(q->level == p->level && q->m == p->m && q->n1 == p->n1 && q->n2 == p->n2 && q->sign == p->sign &&
                  q->span == p->span && q->radix == p->radix,
              "plan %d differs from plan 0 in level, m, n1, n2, sign, radix or fold span", i);
  }
  return HELRM_OK;
}

extern "C" int helrm_footprint_multi(const helrm_ctx *c, const helrm_plan *const *plans, int n_in, int batch,
                                     size_t *bytes) {
  API_GUARD_BEGIN
  TRY(check_multi_plans(c, plans, n_in));
  CHECK_ARG(bytes && batch >= 0, "bad argument");
  *bytes = matvec_ws_bytes(c, plans[0], batch, true, nonzero_giants(plans, n_in));
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_reserve_multi(helrm_ctx *c, const helrm_plan *const *plans, int n_in, int batch,
                                   void *stream) {
  API_GUARD_BEGIN
  TRY(check_multi_plans(c, plans, n_in));
  CHECK_ARG(batch >= 0, "batch < 0");
  char *base;
  return ensure_ws(c, as_stream(stream), matvec_ws_bytes(c, plans[0], batch, true, nonzero_giants(plans, n_in)),
                   &base);
  API_GUARD_END
}

// ---------------------------------------------------------------- captured batch graphs

struct helrm_graph {
  helrm_ctx *ctx = nullptr;
  void *ws = nullptr;             // the graph's own workspace
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" int helrm_batch_graph_destroy(helrm_graph *g) {
  API_GUARD_BEGIN
  if (!g) return HELRM_OK;
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  delete g;
  return HELRM_OK;
  API_GUARD_END
}

// Capture `body` (which enqueues one lookup on the given stream, on the graph's
// own workspace of `bytes`) into g.
template <class F>
int capture_graph(helrm_ctx *c, size_t bytes, F body, helrm_graph **res) {
  helrm_graph *g = new helrm_graph();
  g->ctx = c;
  if (hipMalloc(&g->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    set_error("graph workspace allocation of %zu bytes failed", bytes);
    return HELRM_ENOMEM;
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    helrm_batch_graph_destroy(g);
    set_error("stream creation for the capture failed");
    return HELRM_EHIP;
  }
  int rc = HELRM_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipStreamBeginCapture failed");
    rc = HELRM_EHIP;
  } else {
    rc = body((char *)g->ws, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc == HELRM_OK && e != hipSuccess) {
      set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
      rc = HELRM_EHIP;
    }
    g->graph = graph;
    if (rc == HELRM_OK) {
      const hipError_t ei = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        rc = HELRM_EHIP;
      }
    }
    (void)hipGetLastError();
  }
  (void)hipStreamDestroy(cs);
  if (rc != HELRM_OK) {
    helrm_batch_graph_destroy(g);
    return rc;
  }
  *res = g;
  return HELRM_OK;
}

extern "C" int helrm_batch_graph_create(helrm_ctx *c, const helrm_plan *const *plans, int n_in,
                                        const uint64_t *sel, int batch, uint64_t *out, helrm_graph **res) {
  API_GUARD_BEGIN
  CHECK_ARG(res, "NULL result pointer");
  *res = nullptr;
  TRY(check_multi_plans(c, plans, n_in));
  const helrm_plan *p = plans[0];
  CHECK_ARG(p->level >= 1, "lookup needs plans at level >= 1");
  CHECK_ARG(batch >= 1, "batch must be >= 1");
  CHECK_ARG(sel && out, "NULL buffer");
  CHECK_ARG(!c->timing, "kernel timing is enabled: disable it before capturing a graph");
  const size_t ngu = nonzero_giants(plans, n_in);
  const size_t bytes = matvec_ws_bytes(c, p, batch, true, ngu);
  return capture_graph(c, bytes, [&](char *base, hipStream_t cs) {
    MatvecWS w = carve_matvec(c, p, batch, true, base, ngu);
    const int lv = p->level;
    return run_matvec(c, plans, n_in, sel, n_in * 2 * (lv + 1), w.mv, out, batch, w, cs);
  }, res);
  API_GUARD_END
}

extern "C" int helrm_batch_graph_create_mixed(helrm_ctx *c, const helrm_plan *const *plans, const uint64_t *sel,
                                              int batch, uint64_t *out, helrm_graph **res) {
  API_GUARD_BEGIN
  CHECK_ARG(res, "NULL result pointer");
  *res = nullptr;
  CHECK_ARG(c, "NULL context");
  CHECK_ARG(batch >= 1, "batch must be >= 1");
  CHECK_ARG(sel && out, "NULL buffer");
  CHECK_ARG(!c->timing, "kernel timing is enabled: disable it before capturing a graph");
  std::vector<PlanGroup> groups;
  std::vector<int> order;
  TRY(mixed_groups(c, plans, batch, groups, order));
  CHECK_ARG(groups[0].p->level >= 1, "lookup needs plans at level >= 1");
  return capture_graph(c, mixed_ws_bytes(c, groups, batch), [&](char *base, hipStream_t cs) {
    return lookup_mixed(c, groups, order, sel, batch, out, base, cs);
  }, res);
  API_GUARD_END
}

extern "C" int helrm_batch_graph_replay(helrm_graph *g, void *stream) {
  API_GUARD_BEGIN
  CHECK_ARG(g && g->exec, "NULL or empty graph");
  HIP_TRY(hipGraphLaunch(g->exec, as_stream(stream)));
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_calibrate_alu(helrm_ctx *c, int kind, int prime_index, void *stream, double *per_s) {
  API_GUARD_BEGIN
  CHECK_ARG(c && per_s, "NULL argument");
  CHECK_ARG(kind >= HELRM_CAL_BUTTERFLY && kind <= HELRM_CAL_FMA_F64, "unknown calibration kind %d", kind);
  hipStream_t s = as_stream(stream);
  if (kind == HELRM_CAL_BUTTERFLY) {
    CHECK_ARG(prime_index >= 0 && prime_index < c->nprimes, "prime_index %d out of range", prime_index);
    return calibrate_butterflies(c, c->primes[prime_index], s, per_s);
  }
  return calibrate_instr(kind == HELRM_CAL_MAD_U64 ? 0 : 1, s, per_s);
  API_GUARD_END
}

extern "C" int helrm_timing_enable(helrm_ctx *c, int enable) {
  API_GUARD_BEGIN
  CHECK_ARG(c, "NULL context");
  HIP_TRY(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(c->tmu);
  timing_clear(c);
  c->timing = enable != 0;
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_timing_read(helrm_ctx *c, const char *kernel, double *ms, int64_t *launches, double *bytes,
                                 double *ops) {
  API_GUARD_BEGIN
  CHECK_ARG(c && kernel && ms && launches && bytes && ops, "NULL argument");
  int k = -1;
  for (int i = 0; i < TK_COUNT; i++)
    if (strcmp(kernel, kTimedNames[i]) == 0) k = i;
  CHECK_ARG(k >= 0, "unknown kernel class '%s'", kernel);
  std::lock_guard<std::mutex> lk(c->tmu);
  *ms = 0;
  *launches = 0;
  *bytes = 0;
  *ops = 0;
  for (auto &r : c->trecs) {
    if (r.k != k) continue;
    HIP_TRY(hipEventSynchronize(r.b));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    *ms += t;
    *launches += 1;
    *bytes += r.bytes;
    *ops += r.ops;
  }
  return HELRM_OK;
  API_GUARD_END
}

extern "C" int helrm_set_tuning(helrm_ctx *c, const char *knob, int value) {
  API_GUARD_BEGIN
  CHECK_ARG(c && knob, "NULL argument");
  if (strcmp(knob, "ks_tile") == 0 || strcmp(knob, "baby_tile") == 0) {
    CHECK_ARG(value == 1 || value == 2 || value == 4, "%s must be 1, 2 or 4", knob);
    (knob[0] == 'k' ? c->tune_ks_tile : c->tune_baby_tile) = value;
  } else if (strcmp(knob, "ntt_col_w") == 0) {
    CHECK_ARG(value == 0 || value == 8 || value == 16, "ntt_col_w must be 0, 8 or 16");
    c->tune_ntt_col_w = value;
  } else if (strcmp(knob, "ntt_blk_w") == 0) {
    CHECK_ARG(value == 0 || value == 4 || value == 8, "ntt_blk_w must be 0, 4 or 8");
    c->tune_ntt_blk_w = value;
  } else if (strcmp(knob, "fuse_conv") == 0) {
    CHECK_ARG(value == 0 || value == 1, "fuse_conv must be 0 or 1");
    c->tune_fuse_conv = value;
  } else if (strcmp(knob, "mfma_min_slots") == 0) {
    CHECK_ARG(value >= 0 && value <= 64, "mfma_min_slots must be in 0..64");
    c->tune_mfma_min_slots = value;
  } else if (strcmp(knob, "fold_mp") == 0) {
    CHECK_ARG(value >= 0 && value <= 3, "fold_mp must be 0..3");
    c->tune_fold_mp = value;
  } else if (strcmp(knob, "ks_chain") == 0) {
    CHECK_ARG(value == 0 || value == 1, "ks_chain must be 0 or 1");
    c->tune_ks_chain = value;
  } else if (strcmp(knob, "block_chain") == 0) {
    CHECK_ARG(value == 0 || value == 1, "block_chain must be 0 or 1");
    c->tune_block_chain = value;
  } else if (strcmp(knob, "ntt_small_limbs") == 0) {
    CHECK_ARG(value >= 0, "ntt_small_limbs must be >= 0");
    c->ntt_small_limbs = value;
  } else if (strcmp(knob, "gen_key_a") == 0) {
    CHECK_ARG(value >= 0 && value <= 2, "gen_key_a must be 0, 1 or 2");
    c->tune_gen_key_a = value;
  } else if (strcmp(knob, "limb_xcd") == 0) {
    CHECK_ARG(value == 0 || value == 1, "limb_xcd must be 0 or 1");
    c->tune_limb_xcd = value;
  } else if (strcmp(knob, "fuse_ks") == 0) {
    CHECK_ARG(value == 0 || value == 1, "fuse_ks must be 0 or 1");
    c->tune_fuse_ks = value;
  } else if (strcmp(knob, "conv_wgs") == 0) {
    CHECK_ARG(value >= 0, "conv_wgs must be >= 0");
    c->tune_conv_wgs = value;
  } else if (strcmp(knob, "baby_mfma") == 0) {
    CHECK_ARG(value >= 0, "baby_mfma must be >= 0");
    c->tune_baby_mfma = value;
  } else if (strcmp(knob, "baby_fold") == 0) {
    CHECK_ARG(value >= 0, "baby_fold must be >= 0");
    c->tune_baby_fold = value;
  } else if (strcmp(knob, "ptm") == 0) {
    CHECK_ARG(value == 0 || value == 1, "ptm must be 0 or 1");
    c->tune_ptm = value;
  } else if (strcmp(knob, "baby_share") == 0) {
    CHECK_ARG(value == 1 || value == 2 || value == 4 || value == 8, "baby_share must be 1, 2, 4 or 8");
    c->tune_baby_share = value;
  } else {
    set_error("unknown tuning knob '%s'", knob);
    return HELRM_EINVAL;
  }
  return HELRM_OK;
  API_GUARD_END
}
