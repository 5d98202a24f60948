/*
 * helrm.h -- C ABI of libhelrm, the MI355X (gfx950) library for the CKKS
 * plaintext-matrix x ciphertext-vector product behind HE-LRM's encrypted
 * embedding lookups (arXiv 2506.18150).
 *
 * Paper passages the calls implement:
 *   - Appendix A "CKKS operations": the ring R_Q = Z_Q[X]/(X^N+1) with
 *     Q = q_0 ... q_L, encryption (c0, c1) in R_Q^2, plaintext x ciphertext
 *     multiplication, rescale Q_l -> Q_{l-1}, rotation by k slots, key
 *     switching with a special switching key.
 *   - Sec. II-A "System-Level Costs": rotation needs key switching and one
 *     evaluation key per rotation offset.
 *   - Sec. II-A "Neural Network Layers in FHE" and Sec. III-B "Matrix-Vector
 *     Lookup": y = E^T s computed by the diagonal method with baby-step
 *     giant-step (BSGS) rotations, double-hoisted, consuming one level.
 *   - Sec. IV-B "Block-diagonal embedding matrix" and the end-to-end pipeline:
 *     the server multiplies the packed matrix by the encrypted concatenated
 *     one-hot selector; the result is already packed.
 *
 * Conventions (all calls):
 *   - Residues are uint64, canonical in [0, q).  A polynomial over a basis of
 *     limbs is stored limb-major: limb i occupies N contiguous words.
 *   - Prime indices: 0..L are q_0..q_L, L+1..L+K are the special primes
 *     p_0..p_{K-1}.  A ciphertext at level l has limbs q_0..q_l; an
 *     "extended" (PQ) polynomial at level l has limbs q_0..q_l, p_0..p_{K-1}.
 *   - Ciphertexts are [batch][2][limbs][N] (c0 then c1), in evaluation (NTT)
 *     form: value j of a limb is the polynomial at psi^(2 brv(j)+1) mod q,
 *     brv = log2(N)-bit reversal, psi the root fixed in helrm_create.
 *   - Rotation by k slots (left: slot j receives slot j+k) uses the Galois
 *     element 5^k mod 2N.
 *   - Device pointers named d_* are owned by the caller and must stay valid
 *     until the work enqueued on `stream` has finished.  The library never
 *     frees caller memory.  Keys and plans are copied into library-owned
 *     device memory that lives until helrm_destroy / helrm_plan_destroy.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  Calls
 *     check their arguments on the host, enqueue, and return without
 *     synchronising; only helrm_create, helrm_load_eval_keys and
 *     helrm_plan_create block.  A device-side fault surfaces at the caller's
 *     next synchronisation.
 *   - Calls that need temporaries use a workspace owned by the context, one per
 *     stream, grown on demand (growing synchronises that stream).  Work for
 *     one context on one stream is serialised; different streams get
 *     different workspaces and may overlap.
 *   - An empty call (batch 0, or no limbs or rotations) checks the context
 *     and sizes, may take NULL buffers, enqueues nothing and returns HELRM_OK;
 *     a batch graph needs at least one element (HELRM_EINVAL).
 *   - Return value: HELRM_OK (0) or a negative code; helrm_last_error()
 *     returns a thread-local description of the last failure.  No C++
 *     exception crosses this interface and the library never aborts.
 */
#ifndef HELRM_H
#define HELRM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELRM_OK 0
#define HELRM_EINVAL (-1) /* bad pointer, size, level, basis or missing key */
#define HELRM_ENOMEM (-2) /* device allocation failed */
#define HELRM_EHIP (-3)   /* a HIP runtime call failed */
#define HELRM_ESTATE (-4) /* call not valid in the current state */

typedef struct helrm_ctx helrm_ctx;
typedef struct helrm_plan helrm_plan;

/* RNS-CKKS parameters.  q[0..L] are the ciphertext primes (q_0 is never
 * dropped), p[0..K-1] the special primes of hybrid key switching; every
 * prime is < 2^60 (the lazy integer arithmetic keeps 16 q below 2^64) and
 * = 1 mod 2N.  Key-switching digit j holds the Q primes
 * j*alpha .. j*alpha+alpha-1 (dnum = ceil((L+1)/alpha) digits). */
typedef struct {
  int log_n;            /* N = 2^log_n; 12 or 16 */
  int L;                /* index of the top ciphertext prime */
  int K;                /* number of special primes, 1..16 */
  int alpha;            /* Q primes per digit */
  const uint64_t *q;    /* host, L+1 primes */
  const uint64_t *p;    /* host, K primes */
} helrm_params;

/* Message of the last failing call on this thread ("" if none). */
const char *helrm_last_error(void);

/* Build a context on the current HIP device for the ring R_Q = Z_Q[X]/(X^N+1)
 * with Q = q_0 ... q_L held in residue form (Appendix A "CKKS operations";
 * Sec. II-A "CKKS": ciphertexts are integer polynomials with large
 * coefficients, manipulated with modular arithmetic) and the special primes P
 * of key switching (Appendix A "Key-switching"): per-prime roots psi (from
 * the smallest quadratic non-residue x: psi = x^((q-1)/2N)), twiddle tables
 * and the constants of base conversion, ModDown and rescale.  params and its
 * arrays are read during the call only.  Errors: HELRM_EINVAL (log_n not 12
 * or 16, L/K/alpha out of range, a prime not = 1 mod 2N or not below 2^60, a
 * repeated prime, more than 16 digits), HELRM_ENOMEM, HELRM_EHIP.  Blocks. */
int helrm_create(const helrm_params *params, helrm_ctx **out);
int helrm_destroy(helrm_ctx *ctx);

/* Root psi chosen for prime index i (host query, for checks). */
int helrm_get_psi(const helrm_ctx *ctx, int prime_index, uint64_t *psi);

/* Copy n_keys switching keys into library-owned device memory (Appendix A
 * "Key-switching").  galois[k] is the Galois element of key k (rotation by r
 * slots: 5^r mod 2N); galois 0 denotes the relinearisation key.  `keys`
 * (host or device memory) is [n_keys][dnum][2][L+1+K][N]: for digit j the pair
 * (b_j, a_j) over all L+1+K primes in evaluation form, with
 * b_j = -a_j s + e_j + [P]_{q_i} s' on digit j's primes.  `seeds` (host, may
 * be NULL) gives each key's 64-bit seed when its a_j halves are the seeded
 * uniform polynomials of helrm_key_uniform; kernels that use every key word
 * once (one ciphertext per call) then regenerate a_j instead of reading it,
 * so the caller must pass the seed the a_j were expanded from.  The library
 * holds each key in Montgomery form plus a second copy of the b_j halves on
 * the primes below 2^40 as 40-bit words (5 bytes), which the kernels stream;
 * a key takes dnum (L+1+K) N (16 + 5) bytes.  A key loaded again for the same
 * element replaces the old one.  Blocks. */
int helrm_load_eval_keys(helrm_ctx *ctx, const uint32_t *galois, int n_keys,
                         const uint64_t *keys, const uint64_t *seeds);

/* The uniform half a_j (digit j) of a switching key with the given seed, over
 * all L+1+K primes in evaluation form: out is device [L+1+K][N].  The paper
 * asks only for a uniformly random public polynomial (Appendix A
 * "Encryption", "Key-switching"); this library expands it from a 64-bit seed
 * so that kernels can regenerate it instead of reading it.  Value x on prime
 * index p (counter c = x + 2^16 p + 2^24 j, o_n the n-th output of the
 * SplitMix64 generator of Steele, Lea and Flood, OOPSLA 2014, seeded with
 * `seed`) is (X mod q_p) 2^-128 mod q_p, where X = o_{2c+2} 2^64 + o_{2c+1}
 * when q_p >= 2^40 (within 2^-68 of uniform), and when q_p < 2^40 X is the
 * first of o_{2c+1}, o_{2^32+4c+1}, o_{2^32+4c+2}, o_{2^32+4c+3} below
 * 2^64 - (2^64 mod q_p) (rejection sampling: uniform but for a 2^-96 tail).
 * Errors: HELRM_EINVAL (digit out of range, NULL out). */
int helrm_key_uniform(helrm_ctx *ctx, uint64_t seed, int digit, uint64_t *out, void *stream);

/* Forward / inverse negacyclic NTT, in place, of `batch` blocks of n_limbs
 * limbs each (block b at d_data + b*n_limbs*N); limb i of every block uses
 * prime prime_index[i] (host array).  Forward maps coefficients to evaluation
 * form as defined above; inverse is its exact inverse (includes N^-1).  The
 * paper's polynomial products in R_Q (Appendix A "Multiplication"; Sec. II-A
 * "CKKS") become slot-wise products in this form, which every other call
 * works in.  Errors: HELRM_EINVAL (NULL buffer, prime index out of range,
 * negative size). */
int helrm_ntt(helrm_ctx *ctx, uint64_t *d_data, int n_limbs, const int32_t *prime_index,
              int batch, void *stream);
int helrm_intt(helrm_ctx *ctx, uint64_t *d_data, int n_limbs, const int32_t *prime_index,
               int batch, void *stream);

/* Automorphism X -> X^galois in evaluation form (a permutation of each limb):
 * d_out[j] = d_in[j'] with 2 brv(j')+1 = galois (2 brv(j)+1) mod 2N.  With
 * galois = 5^k mod 2N it is the slot rotation by k of Appendix A "Rotation"
 * before its key switch (the result decrypts under sigma(s)).  galois must
 * be odd.  d_in and d_out must not overlap.  Layout [batch][n_limbs][N].
 * Errors: HELRM_EINVAL (even or out-of-range galois, NULL or equal buffers). */
int helrm_automorph(helrm_ctx *ctx, const uint64_t *d_in, uint64_t *d_out, uint32_t galois,
                    int n_limbs, int batch, void *stream);

/* Element-wise arithmetic over [batch][n_limbs][N] (limb i uses prime
 * prime_index[i]).  op: 0 add, 1 sub (a - b), 2 mul, 3 neg (b ignored).
 * Outputs may alias inputs. */
#define HELRM_OP_ADD 0
#define HELRM_OP_SUB 1
#define HELRM_OP_MUL 2
#define HELRM_OP_NEG 3
int helrm_poly_op(helrm_ctx *ctx, int op, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out,
                  int n_limbs, const int32_t *prime_index, int batch, void *stream);

/* d_out[b][i][j] = d_a[b][i][j] * scalars[i] mod q (scalars: host, one per limb). */
int helrm_mul_scalar(helrm_ctx *ctx, const uint64_t *d_a, const uint64_t *scalars, uint64_t *d_out,
                     int n_limbs, const int32_t *prime_index, int batch, void *stream);

/* Signed integer coefficients to residues: d_out[b][i][j] = d_in[b][j] mod q
 * (d_in: device int64 [batch][N]; coefficient form, no NTT applied). */
int helrm_from_signed(helrm_ctx *ctx, const int64_t *d_in, uint64_t *d_out, int n_limbs,
                      const int32_t *prime_index, int batch, void *stream);

/* Hoisted rotations with key switching (Appendix A "Rotation",
 * "Key-switching"; hoisting as in the double-hoisted BSGS of Sec. III-B).
 * One ModUp of c1 (digit decomposition + fast base conversion to the extended
 * basis, uncorrected), then for each step k: the automorphism of every digit,
 * the inner product with the key of 5^k, plus P * sigma(c0):
 *   A = sum_j sigma(d_j) a_j,  B = sum_j sigma(d_j) b_j + P sigma(c0).
 * d_ct: [batch][2][level+1][N].  out_basis 0 (Q): each output is divided by P
 * (ModDown, no rounding offset) -> d_out [batch][n_rot][2][level+1][N], a
 * rotated ciphertext.  out_basis 1 (PQ): kept as (B, A) over the extended
 * basis -> d_out [batch][n_rot][2][level+1+K][N].  Keys for every step must
 * be loaded; step 0 is allowed and gives (P c0, P c1) (PQ) or the input (Q). */
#define HELRM_BASIS_Q 0
#define HELRM_BASIS_PQ 1
int helrm_keyswitch_hoisted(helrm_ctx *ctx, const uint64_t *d_ct, int level,
                            const int32_t *rot_steps, int n_rot, uint64_t *d_out,
                            int out_basis, int batch, void *stream);

/* Rescale Q_l -> Q_{l-1} (Appendix A "Multiplication"): each coefficient C
 * (CRT value in [0, Q_l)) becomes floor((C + floor(q_l/2)) / q_l) mod Q_{l-1}.
 * d_in [batch][2][level+1][N] -> d_out [batch][2][level][N].  level >= 1. */
int helrm_rescale(helrm_ctx *ctx, const uint64_t *d_in, int level, uint64_t *d_out, int batch,
                  void *stream);

/* A plaintext matrix prepared for the BSGS diagonal method (Sec. II-A
 * "Neural Network Layers in FHE", Sec. III-B).  For an r x c matrix M (r
 * outputs, c <= N/2 inputs) with m = next power of two >= r and a direction
 * sign = +1 or -1, the hybrid diagonals are
 * u_k[j] = M[j mod m][(j + sign*k) mod (N/2)] (zero rows beyond r), k < m.
 * With k = n1*g + b, the plan holds v_{g,b} = rot(u_k, -sign*n1*g) encoded at
 * scale q_level as signed integer coefficients.  The product is
 *   z = sum_g rot( sum_b v_{g,b} (.) rot(x, sign*b), sign*n1*g ),
 * followed by a fold from `fold_span` slots down to period m: each stage with
 * stride s and radix r replaces z by sum_{t<r} rot(z, t*s) (s = span/r,
 * r = min(radix, span/m), span starting at fold_span).  Slot i < r then holds
 * (M x)_i.  With sign = +1 the fold must cover all N/2 slots; with sign = -1
 * every partial sum lies in [0, c + m - 1), so any power of two >= c + m - 1
 * is a valid fold_span. */
typedef struct {
  int level;              /* level of the input ciphertext */
  int m;                  /* number of hybrid diagonals (power of two) */
  int n1;                 /* baby steps */
  int n2;                 /* giant steps, n1*n2 >= m */
  int radix;              /* fold radix >= 2 */
  int n_diag;             /* number of non-zero diagonals given */
  const int32_t *diag;    /* host [n_diag]: k = n1*g + b of each diagonal, ascending */
  const int64_t *coeffs;  /* host [n_diag][N]: coefficients of v_{g,b} at scale q_level */
  int sign;               /* +1 or -1: direction of the baby and giant rotations */
  int fold_span;          /* power of two in [m, N/2]; 0 means N/2 */
} helrm_plan_desc;

/* Reduce the plan's coefficients over the extended basis at its level, take
 * them to evaluation form on the device and keep them resident, each word
 * also as a 40-bit value (the per-ciphertext baby-step kernel streams the
 * limbs of primes below 2^40 in 5 bytes): n_diag (level+1+K) N (8 + 5)
 * bytes.  Blocks. */
int helrm_plan_create(helrm_ctx *ctx, const helrm_plan_desc *desc, helrm_plan **out);
int helrm_plan_destroy(helrm_plan *plan);

/* Fold the evaluation keys into the plan's plaintext diagonals for batched
 * lookups (the product of Sec. III-B reassociated: sum_b pt_b sum_j
 * sigma_b(d_j) k_{b,j} = sum_{b,j} sigma_b(d_j) (pt_b k_{b,j}), identical
 * residues): the library builds and keeps W = pt_{g,b} k_{b,j} (and pt P for
 * the c0 terms) as matrix-core operands, and lookups of at least `baby_fold`
 * ciphertexts (helrm_set_tuning, default 8) then form no rotated ciphertext
 * at all.  Needs the keys of every baby step loaded; a later
 * helrm_load_eval_keys makes the folded words stale (lookups then use the
 * other kernels until the plan is folded again).  Memory: per giant tile of
 * 8, (level+1+K) N ceil(4 n_baby / 64) KiB times 5 (primes below 2^40) or 8
 * digits; *bytes (may be NULL) receives the total.  At most 3 key-switching
 * digits.  Blocks.  Errors: HELRM_EINVAL (foreign plan, missing key, more than
 * 3 digits), HELRM_ENOMEM. */
int helrm_plan_fold_keys(helrm_ctx *ctx, helrm_plan *plan, size_t *bytes);

/* Galois steps the plan needs keys for (host query): writes up to `cap`
 * rotation steps into steps and their count into *n. */
int helrm_plan_rotation_steps(const helrm_plan *plan, int32_t *steps, int cap, int *n);

/* Double-hoisted BSGS plaintext-matrix x ciphertext product without rescale:
 *   1. ModUp(c1) once; R_0 = (P c0, P c1); R_b = hoisted rotation by sign*b (PQ).
 *   2. X_g = sum_b pt_{g,b} (.) R_b over PQ; x_g = ModDown(X_g).
 *   3. acc = P x_0 + sum_{g>=1} (rotation of x_g by sign*n1*g, kept in PQ);
 *      z = ModDown(acc)  (z = x_0 when only g = 0 has diagonals).
 *   4. Fold: per stage (s, r): z = ModDown(P z + sum_{t=1}^{r-1} rot_PQ(z, t s)).
 * d_ct [batch][2][level+1][N] -> d_out [batch][2][level+1][N] at scale
 * (input scale * q_level). */
int helrm_ptxt_ct_matvec_diag(helrm_ctx *ctx, const helrm_plan *plan, const uint64_t *d_ct,
                              uint64_t *d_out, int batch, void *stream);

/* Encrypted packed embedding lookup (Sec. IV-B pipeline): the matvec above
 * followed by rescale, so the result is at level-1 and at the selector's
 * scale.  d_sel [batch][2][level+1][N] -> d_out [batch][2][level][N]; table t's
 * row lands in slots [d*t, d*t + d) when the plan packs tables block-diagonally. */
int helrm_lookup_packed(helrm_ctx *ctx, const helrm_plan *plan, const uint64_t *d_sel,
                        int batch, uint64_t *d_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * lookup as helrm_lookup_packed, same arguments, layouts, kernels and results,
 * but its workspace is a static device array of HELRM_NOALLOC_MAX_BYTES per
 * GPU (held from the first helrm_create on that GPU until the process ends)
 * instead of the stream's workspace.  It allocates nothing (no hipMalloc, no
 * hipFree, no allocating library call) and never synchronises.  The caller
 * still owns d_sel and d_out.  The call must be made with the context's
 * device current.  Every call on one GPU, from any context or stream, shares
 * that GPU's array and finds it holding the previous call's contents (no part
 * of the workspace needs to start at zero): calls that overlap in time on one
 * GPU race and corrupt each other's results, so serialise them (one stream, or
 * events).  Errors: HELRM_EINVAL (as helrm_lookup_packed; a call whose
 * helrm_footprint exceeds HELRM_NOALLOC_MAX_BYTES, e.g. level 23 at N=2^16;
 * kernel timing enabled; wrong current device), HELRM_EHIP. */
#define HELRM_NOALLOC_MAX_BYTES (256ull << 20)
int helrm_lookup_packed_noalloc(helrm_ctx *ctx, const helrm_plan *plan, const uint64_t *d_sel,
                                int batch, uint64_t *d_out, void *stream);

/* Device bytes one call of helrm_lookup_packed with this batch uses beyond its
 * input and output (workspace), for admission control. */
int helrm_footprint(const helrm_ctx *ctx, const helrm_plan *plan, int batch, size_t *bytes);

/* Grow the workspace of `stream` to serve helrm_lookup_packed(plan, batch)
 * without further allocation (call before capturing a graph).  A call that
 * needs a larger workspace while its stream is being captured fails with
 * HELRM_ESTATE instead of allocating; a workspace that a capture has used is
 * kept (not freed) when a later eager call outgrows it, so graphs captured on
 * it stay valid until helrm_destroy. */
int helrm_reserve(helrm_ctx *ctx, const helrm_plan *plan, int batch, void *stream);

/* Give back the workspace of `stream` (for callers that retire a stream, such
 * as a serving executor that is replaced): waits for the stream, then frees
 * its workspace; a workspace that a graph capture used is kept until
 * helrm_destroy instead, since the graph may still be replayed.  A later call
 * on the stream allocates afresh.  No-op for a stream without a workspace.
 * Errors: HELRM_ESTATE while the stream is being captured, HELRM_EHIP. */
int helrm_release_stream(helrm_ctx *ctx, void *stream);

/* helrm_footprint / helrm_reserve for helrm_lookup_multi: the workspace of
 * one call with these plans (the same checks as helrm_lookup_multi), which
 * also holds the ModUp digits of every giant step in the union of the plans'.
 * Errors: HELRM_EINVAL (mismatched plans), HELRM_ENOMEM. */
int helrm_footprint_multi(const helrm_ctx *ctx, const helrm_plan *const *plans, int n_in, int batch,
                          size_t *bytes);
int helrm_reserve_multi(helrm_ctx *ctx, const helrm_plan *const *plans, int n_in, int batch, void *stream);

/* A batch of lookups over uneven packings: element b of the batch goes
 * through plans[b] (the encrypted packed lookup of Sec. IV-B, each element with
 * its own block-diagonal packing, e.g. its own subset of tables).  The plans
 * share the context, the level, n1 and the rotation direction, and either all
 * or none have giant steps beyond g = 0; their diagonals, giant steps and fold
 * spans may differ.  The steps that do not depend on the plan (ModUp,
 * the ModDown boundaries, the rescale) run once over the whole batch; the
 * baby-step MAC and the key-switch accumulations run once per distinct plan.
 * Results are the same residues as helrm_lookup_packed with each element's
 * plan.  d_sel [batch][2][level+1][N] -> d_out [batch][2][level][N], both
 * caller-owned; plans is a host array of batch plan pointers, read during the
 * call.  Errors: HELRM_EINVAL (NULL or foreign plan, plans that differ in
 * level, n1, direction or in having giant steps), HELRM_ENOMEM,
 * HELRM_ESTATE (the stream's workspace would grow during capture). */
int helrm_lookup_batch(helrm_ctx *ctx, const helrm_plan *const *plans, const uint64_t *d_sel, int batch,
                       uint64_t *d_out, void *stream);
/* Workspace of one helrm_lookup_batch call with these plans, and its
 * reservation on `stream` (as helrm_footprint / helrm_reserve). */
int helrm_footprint_batch(const helrm_ctx *ctx, const helrm_plan *const *plans, int batch, size_t *bytes);
int helrm_reserve_batch(helrm_ctx *ctx, const helrm_plan *const *plans, int batch, void *stream);

/* A batch of lookups captured once as a HIP graph and replayed (the batched
 * form of the Sec. IV-B pipeline: every ciphertext of the batch goes through
 * the same plan, so the whole launch sequence of helrm_lookup_packed, or of
 * helrm_lookup_multi when n_in > 1, is fixed and replays as one graph launch).
 * helrm_batch_graph_create records lookup(plans, d_sel, batch, d_out) on a
 * stream of its own (nothing runs), with a workspace the graph owns
 * (helrm_footprint_multi bytes, allocated here).  d_sel
 * ([batch][n_in][2][level+1][N]) and d_out ([batch][2][level][N]) are bound
 * to the graph: the caller writes the next selectors into d_sel and calls
 * helrm_batch_graph_replay, which enqueues the recorded launches on `stream`
 * and returns.  d_sel, d_out, the plans and the context's keys must stay
 * valid until helrm_batch_graph_destroy (which waits for the device).
 * Replays on different streams must not overlap (they share the workspace).
 * Errors: HELRM_EINVAL (mismatched plans, batch < 1, NULL buffer, missing
 * key), HELRM_ESTATE (kernel timing enabled while capturing), HELRM_ENOMEM,
 * HELRM_EHIP. */
typedef struct helrm_graph helrm_graph;
int helrm_batch_graph_create(helrm_ctx *ctx, const helrm_plan *const *plans, int n_in, const uint64_t *d_sel,
                             int batch, uint64_t *d_out, helrm_graph **out);
/* The same for a batch over uneven packings (plans[b] for element b, as
 * helrm_lookup_batch): one captured launch sequence, replayed with
 * helrm_batch_graph_replay. */
int helrm_batch_graph_create_mixed(helrm_ctx *ctx, const helrm_plan *const *plans, const uint64_t *d_sel,
                                   int batch, uint64_t *d_out, helrm_graph **graph);
int helrm_batch_graph_replay(helrm_graph *graph, void *stream);
int helrm_batch_graph_destroy(helrm_graph *graph);

/* ALU ceilings for the rooflines of the integer-bound kernels (measurement
 * only, not part of any lookup).  kind HELRM_CAL_BUTTERFLY: butterflies per
 * second of the NTT's arithmetic on prime `prime_index` (the policy its
 * transforms use: fp64 exact products below 2^41, Shoup products above),
 * every thread repeating radix-16 butterfly phases on registers with no
 * memory traffic; HELRM_CAL_MAD_U64: 32x32->64 integer multiply-adds per
 * second (per lane), the instruction every modular product of the library
 * is built from; HELRM_CAL_FMA_F64: fp64 FMAs per second (per lane).  Runs
 * on `stream` after one warm-up launch, allocates a small buffer, blocks.
 * Errors: HELRM_EINVAL (unknown kind, prime index out of range), HELRM_EHIP. */
#define HELRM_CAL_BUTTERFLY 0
#define HELRM_CAL_MAD_U64 1
#define HELRM_CAL_FMA_F64 2
int helrm_calibrate_alu(helrm_ctx *ctx, int kind, int prime_index, void *stream, double *per_s);

/* Kernel timing for measurement.  While enabled, every launch of the timed
 * kernel classes records a pair of HIP events on its stream (enabling or
 * disabling synchronises the device and clears earlier records).  Classes:
 * "ntt_fwd_col", "ntt_fwd_blk", "ntt_inv_blk", "ntt_inv_col" (the two passes
 * of each transform), "conv" (fast base conversion), "ks_acc" (key inner
 * product + automorphism), "baby_mac" (fused baby steps and plaintext MAC),
 * "sub_mul" (ModDown / rescale finish), "baby_mfma" (the same on the matrix
 * cores) and "baby_fold" (the key-folded product and its entries pass).  helrm_timing_read waits for the
 * recorded launches of one class and returns their summed duration (ms), the
 * launch count, and the bytes and modular products those launches process
 * (every operand read once, every result written once; for the matrix-core
 * classes the bytes those kernels stream, see the kernel notes). */
int helrm_timing_enable(helrm_ctx *ctx, int enable);
int helrm_timing_read(helrm_ctx *ctx, const char *kernel, double *ms, int64_t *launches, double *bytes,
                      double *ops);

/* Lookup for a packed selector wider than one ciphertext (Sec. III-C: a
 * selector of k slots needs ceil(k / n) ciphertexts): ciphertext c carries
 * slots [c n, (c+1) n) and plans[c] holds the diagonals of the matching column
 * block of M.  The plans must share level, m, n1, n2, rotation direction, fold
 * radix and fold span; every block's baby-step products are summed into the
 * same giant-step accumulators, after which the giant steps, the fold and the
 * rescale run once, so out = Enc(sum_c M_c s_c) at level-1.  sel: device
 * [batch][n_in][2][level+1][N]; out: device [batch][2][level][N].  Workspace as
 * helrm_footprint of plans[0] (plus the digits of every giant step in the
 * union of the plans').  Errors: HELRM_EINVAL (mismatched plans, missing key),
 * HELRM_ENOMEM. */
int helrm_lookup_multi(helrm_ctx *ctx, const helrm_plan *const *plans, int n_in, const uint64_t *sel, int batch,
                       uint64_t *out, void *stream);

/* Ciphertext-ciphertext product with relinearisation (Appendix A
 * "Multiplication", "Key-switching"): the tensor product
 * (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) followed by a hybrid key switch
 * of d2 from s^2 to s with the relinearisation key (loaded as Galois element
 * 0): ModUp(d2), inner product with the key plus P (d0, d1), ModDown.  No
 * rescale (call helrm_rescale).  a, b, out: device [batch][2][level+1][N] in
 * evaluation form; a may equal b (square) and out may alias a or b.  Errors:
 * HELRM_EINVAL (level, NULL buffer, no relinearisation key). */
int helrm_mul_relin(helrm_ctx *ctx, const uint64_t *a, const uint64_t *b, int level, uint64_t *out, int batch,
                    void *stream);

/* Plaintext-ciphertext addition (Appendix A "Addition"): out = (c0 + pt, c1)
 * for every ciphertext of the batch.  ct, out: device [batch][2][level+1][N];
 * pt: device [level+1][N] residues in evaluation form (the plaintext encoded at
 * the ciphertext's scale), shared by the batch; out may alias ct.  Errors:
 * HELRM_EINVAL. */
int helrm_add_plain(helrm_ctx *ctx, const uint64_t *ct, const uint64_t *pt, int level, uint64_t *out,
                    int batch, void *stream);

/* Level alignment without rescaling: the same ciphertext modulo Q_level_out
 * (limbs above q_level_out dropped), so that ciphertexts of different depths
 * can be added.  in: device [batch][2][level_in+1][N]; out: device
 * [batch][2][level_out+1][N], distinct from in.  Errors: HELRM_EINVAL. */
int helrm_mod_drop(helrm_ctx *ctx, const uint64_t *in, int level_in, uint64_t *out, int level_out, int batch,
                   void *stream);

/* Schedule knobs set by the autotuner.  "ks_tile" and "baby_tile" cap how many
 * ciphertexts of a batch one thread serves in the key inner product and the
 * fused baby-step kernel (1, 2 or 4; default 4): larger tiles read each key
 * and plaintext word fewer times, smaller tiles use fewer registers.
 * "baby_share" (1, 2, 4 or 8; default 8) is the number of ciphertexts one
 * workgroup of the fused baby-step kernel serves when a launch has several
 * giant outputs and a batch (each plaintext word is then read once per that
 * many ciphertexts); 1 turns that kernel off.  "ntt_col_w" (8 or 16, default
 * 16) and "ntt_blk_w" (4 or 8, default 4) are the sub-transforms per workgroup
 * of the NTT's column and block passes; 0 picks the narrow shape for launches
 * of fewer than "ntt_small_limbs" limbs (default 48).  Results do not depend
 * on the knobs.  "gen_key_a" lets kernels that use every key word once
 * regenerate seeded keys' a_j halves instead of reading them: 0 never, 1
 * (default) on primes below 2^40, 2 on every prime.
 * "ks_chain" (1, default, or 0): the key-switching kernels take their
 * coefficient blocks in the order in which the rotations shift them, each XCD
 * an eighth of every limb (rotated words then come from L2).  With 0,
 * "limb_xcd" (0, default, or 1): the key-switching kernels deal coefficient
 * blocks over all 8 XCDs, or give each XCD whole limbs (a limb's rotated words
 * are then re-read from one L2: less HBM traffic, less even load).  "fuse_ks" (1, default, or 0): a
 * ModDown feeding a ModUp or the rescale runs fused with it in coefficient
 * form.  "fuse_conv" (1, default, or 0): in such a fused boundary c1's
 * ModDown runs inside the ModUp conversions (one conversion launch instead
 * of two).  "conv_wgs" (>= 0, default 1536): a base conversion launch with fewer
 * workgroups than this splits its outputs into chunks (at least four outputs
 * each) until it has that many; 0 never splits.  "baby_mfma" (>= 0, default
 * 8): batches of at least this many ciphertexts run the plaintext MAC of the
 * baby steps on the matrix cores (0: never), for plans with at least
 * "mfma_min_slots" (0..64, default 33) baby steps (b = 0 included).  "baby_fold" (>= 0, default 8):
 * batches of at least this many use a plan's folded keys
 * (helrm_plan_fold_keys; 0: never).  "ptm" (1, default, or 0): plans keep the
 * plaintexts' matrix-core operands (only plans created while their baby-step
 * count is at least "mfma_min_slots": the others would never use them).  "block_chain" (1, default, or 0): the
 * key-folded product takes its coefficient blocks in the order in which the
 * baby-step rotations shift them (rotated words then come from L2), or in
 * plain order.  "fold_mp" (0..3, default 2): batches of more than 16
 * ciphertexts let one load of the folded operands serve two tiles of 16
 * ciphertexts on primes below 2^40 (bit 0) and on the wider ones (bit 1).
 * Errors: HELRM_EINVAL for an unknown knob or value. */
int helrm_set_tuning(helrm_ctx *ctx, const char *knob, int value);

#ifdef __cplusplus
}
#endif
#endif /* HELRM_H */
