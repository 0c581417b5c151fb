/*
 * rbk.h -- C ABI of librbk: RNS-CKKS ciphertext arithmetic on AMD gfx950.
 *
 * The operations are those ReBoot trains its encrypted MLPs with (paper
 * Section 3): the parameter set {N, q, Delta}, slot-wise add / sub / mult
 * (eqs. add, sub, mult), plaintext-ciphertext ops, the rotation Rot(a, k)
 * with one key per index, and rescaling ("switching to the next prime").
 * The multiplication is relinearised with hybrid key switching (Han-Ki 2020)
 * and rotations are Galois automorphisms X -> X^(5^k).
 *
 * Memory model
 *  - Every `d_` pointer is DEVICE memory owned by the caller (PyTorch in the
 *    Python binding); every other pointer is host memory owned by the caller.
 *    The library never frees caller memory.
 *  - A ciphertext at level l is `uint64_t[2][l+1][N]`, a plaintext
 *    `uint64_t[l+1][N]`; limb i holds residues modulo q_i, canonical in
 *    [0, q_i).  Batched calls take `count` of them back to back.  Device
 *    buffers start on a 16-byte boundary (the kernels move adjacent residue
 *    pairs; device allocations are 256-byte aligned).
 *  - Device ciphertexts and plaintexts are in the NTT (evaluation) domain:
 *    limb i of the transform of a(X) holds a(psi_i^(2k+1)) at index
 *    bit_reverse(k), psi_i the smallest primitive 2N-th root modulo q_i.
 *    rbk_ntt converts; host-side import/export uses the coefficient domain.
 *  - Key material (secret, public key, relinearisation and Galois keys)
 *    lives in device memory owned by the context.
 *  - Calls are asynchronous on the context's stream unless they return host
 *    data (rbk_decode, rbk_key_export, rbk_moduli...), which synchronise.
 *    Device inputs must stay valid until the stream reaches the call.
 *  - A context is not thread-safe.  Scales are tracked by the caller: these
 *    functions only transform residues, except the *_scaled additions (which
 *    check them), the bootstrap (which returns its output scale) and the MLP
 *    (which keeps each state ciphertext's scale).
 *
 * Errors: 0 on success, else a negative RBK_E* code; rbk_last_error()
 * returns a message for the calling thread.  No C++ exception crosses the ABI.
 */
#ifndef RBK_H
#define RBK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBK_OK 0
#define RBK_EINVAL (-1)      /* bad argument or shape */
#define RBK_ENOMEM (-2)      /* host or device allocation failed */
#define RBK_ELEVEL (-3)      /* level out of range for the operation */
#define RBK_ENOKEY (-4)      /* secret, public, relinearisation or Galois key missing */
#define RBK_EDEVICE (-5)     /* HIP runtime error */
#define RBK_ESTATE (-6)      /* operation needs state that is not set up */
#define RBK_EUNSUPPORTED (-7)
#define RBK_ESCALE (-8)      /* operands of an addition at different scales */

typedef struct rbk_ctx rbk_ctx;

/* Parameters Theta = {N, q, Delta} of Section 3, in RNS form.
 *  log_n  : N = 2^log_n, 4 <= log_n <= 17
 *  n_q    : number of primes of the modulus chain q_0..q_{n_q-1}; the top
 *           level is L = n_q - 1 and each rescale drops the last prime
 *  q_bits : bit size of each q_i (log_n+2 .. 60)
 *  n_p    : number of special primes p_0..p_{n_p-1} of key switching
 *  p_bits : their bit sizes
 *  alpha  : primes per key-switching digit (1..16); the number of digits at
 *           level l is ceil((l+1)/alpha)
 * Primes: for each requested size b, in the order q_bits then p_bits, the
 * first q = 2^b - j*2N + 1 (j = 1, 2, ...) that is prime and not yet taken. */
typedef struct {
    uint32_t log_n;
    uint32_t n_q;
    const uint32_t *q_bits;
    uint32_t n_p;
    const uint32_t *p_bits;
    uint32_t alpha;
} rbk_params;

/* ---- context ------------------------------------------------------------ */

/* Create a context on the current HIP device: finds the primes, builds the
 * NTT and base-conversion tables in device memory.  *out owned by caller,
 * released with rbk_ctx_destroy. */
int rbk_ctx_create(const rbk_params *params, rbk_ctx **out);
int rbk_ctx_destroy(rbk_ctx *ctx);
/* Stream (hipStream_t, may be NULL for the default stream) for later calls. */
int rbk_set_stream(rbk_ctx *ctx, void *hip_stream);
int rbk_sync(rbk_ctx *ctx);
const char *rbk_last_error(void);
/* host out[n_q + n_p]: q_0..q_{n_q-1}, p_0..p_{n_p-1} */
int rbk_moduli(const rbk_ctx *ctx, uint64_t *out);
/* host out[n_q + n_p]: the psi of each prime */
int rbk_psi(const rbk_ctx *ctx, uint64_t *out);
/* number of key-switching digits at `level` (>= 0 on success) */
int rbk_num_digits(const rbk_ctx *ctx, int level);
/* Pre-size the device workspace for `count` ciphertexts at `level` doing
 * hoisted rotations (optional; calls grow it on demand otherwise). */
int rbk_reserve(rbk_ctx *ctx, int level, int count);
/* Words of workspace that batched calls on `count` ciphertexts at `level`
 * need: mult_relin, rescale and a hoisted batch of n_rot rotations with the
 * current lane setting. */
int rbk_workspace_words(const rbk_ctx *ctx, int level, int count, int n_rot, size_t *words);
/* The context's workspace (key-switching scratch of every call) becomes the
 * caller's device buffer d_ws of `words` 64-bit words: the caller owns it,
 * keeps it alive and leaves it alone while calls are in flight; a call that
 * needs more returns RBK_ENOMEM instead of allocating.  Synchronises with
 * the context stream, releases a library-owned workspace; d_ws = NULL with
 * words = 0 returns to a library-owned one.  The lanes' scratch, bootstrap
 * registers, MLP buffers and descriptor arenas keep their own allocations.
 * RBK_ESTATE during graph capture. */
int rbk_set_workspace(rbk_ctx *ctx, uint64_t *d_ws, size_t words);

/* ---- transforms --------------------------------------------------------- */

/* In-place forward (inverse = 0) or inverse NTT of d_data[count][n_limbs][N];
 * limb i of every polynomial uses the prime with table index prime_idx[i]
 * (host array; 0..n_q-1 are Q primes, n_q.. the special primes).  The index
 * list must be a run of Q primes 0..a-1 optionally followed by a run of
 * consecutive special primes starting at p_0, or a run of special primes.
 * Inputs are residues in [0, q) (as every residue of this API); outputs are
 * in [0, q).  Residues outside [0, q) give unspecified results. */
int rbk_ntt(rbk_ctx *ctx, uint64_t *d_data, int count, const int *prime_idx, int n_limbs, int inverse);

/* ---- keys (Section 3: sk/pk; rotation keys, one per index) -------------- */
/* These calls take every random input from the caller, so that the same
 * draws can be replayed elsewhere (rbk_keygen below draws them itself).
 * All host arrays, coefficient domain. */

/* s[N]: secret key coefficients (ternary). */
int rbk_set_secret(rbk_ctx *ctx, const int64_t *s);
/* pk = (-a s + e, a) over q_0..q_{n_q-1}; a[n_q][N] uniform residues, e[N]. */
int rbk_keygen_public(rbk_ctx *ctx, const uint64_t *a, const int64_t *e);
/* Relinearisation key (switches s^2 -> s).  beta = ceil(n_q/alpha) digits;
 * a[beta][n_q+n_p][N] uniform residues, e[beta][N] errors.  Digit j:
 *   b_j = -a_j s + e_j + [P]_{q_i} s'  mod q_i for q_i in digit j,
 *   b_j = -a_j s + e_j                  for every other prime. */
int rbk_keygen_relin(rbk_ctx *ctx, const uint64_t *a, const int64_t *e);
/* Key for the automorphism X -> X^g (g odd, < 2N): switches sigma_g(s) -> s.
 * Same randomness layout as rbk_keygen_relin. */
int rbk_keygen_galois(rbk_ctx *ctx, uint64_t g, const uint64_t *a, const int64_t *e);
/* Galois element of a left rotation by k slots: 5^(k mod N/2) mod 2N;
 * conjugation is 2N-1. */
uint64_t rbk_galois_elt(const rbk_ctx *ctx, int64_t k);
/* Copy a key to the host, coefficient domain, [beta][2][n_q+n_p][N]
 * (g = 0 selects the relinearisation key). */
int rbk_key_export(rbk_ctx *ctx, uint64_t g, uint64_t *out);

/* ---- keys and encryption from one seed (seeded sampling) ---------------- */
/* The randomness of Section 3's key generation and encryption (secret,
 * uniform public polynomials, added noise) drawn inside the library from a
 * 64-bit seed, so a client needs no random source of its own.  Keystream:
 * the ChaCha20 block function of RFC 8439 with key (seed low 32 bits, seed
 * high 32 bits, 0 x 6), block counter, nonce (purpose, id, sub):
 *   secret, uniform ternary   (1, 0, 0); exactly h non-zeros: (1, 1, 0)
 *   public key a limb t / e   (2, 0, t) / (3, 0, 0)
 *   switching key, element g (0 = relinearisation), digit j:
 *                 a limb t    (4, g, j * 2^16 + t);  e  (5, g, j)
 *   encryption number i       v (6, i_lo, i_hi), e0 (7, ...), e1 (8, ...)
 * Coefficient j of a polynomial reads the block at counter j (then j + N,
 * j + 2N, ... if that block gives no value): uniform mod q = the first of
 * its eight little-endian 64-bit words, masked to bitlen(q) bits, that is
 * below q; ternary = the first of its 256 2-bit fields (low bits of word 0
 * first) that is not 3, with 0, 1, 2 -> 0, +1, -1; Gaussian (sigma = 3.2,
 * |x| <= 19) = the least m with (w >> 1) < T[m], w the first 64-bit word,
 * T[m] = floor(2^63 P(|x| <= m)) (T[19] = 2^63), negative when m > 0 and
 * bit 0 of w is set.  Secret with h non-zeros: 32-bit stream words in
 * counter order, two per draw, position = first & (N-1), sign = bit 0 of the
 * second (set: -1), taken positions skipped, until h are set. */

/* Secret (uniform ternary when secret_hw = 0, else exactly secret_hw
 * non-zeros), public key, relinearisation key and one Galois key for each
 * rotation step in rot_steps[n_rot] (host) plus the conjugation when conj is
 * non-zero; repeated elements and steps that are multiples of N/2 are
 * skipped.  Replaces keys of the same elements.  Synchronises. */
int rbk_keygen(rbk_ctx *ctx, uint64_t seed, int secret_hw, const int64_t *rot_steps, int n_rot, int conj);
/* rbk_encrypt with (v, e0, e1) drawn from (seed, index).  Asynchronous. */
int rbk_encrypt_seeded(rbk_ctx *ctx, const uint64_t *d_pt, int level, uint64_t seed, uint64_t index, uint64_t *d_ct);
/* host out[20]: the cumulative table T of the Gaussian sampler. */
int rbk_gauss_table(uint64_t *out);

/* ---- ciphertext export / import ---------------------------------------- */
/* Copy npoly polynomials at `level` (a ciphertext: npoly = 2) between device
 * memory (NTT domain) and host memory (coefficient domain,
 * [npoly][level+1][N] canonical residues).  Export synchronises; import
 * checks every residue (RBK_EINVAL if one is not below its prime; d_ct is
 * then unspecified) and transforms d_ct in place. */
int rbk_ct_export(rbk_ctx *ctx, const uint64_t *d_ct, int level, int npoly, uint64_t *out);
int rbk_ct_import(rbk_ctx *ctx, const uint64_t *in, int level, int npoly, uint64_t *d_ct);

/* ---- encoding and encryption ------------------------------------------- */

/* Encode n <= N/2 complex slot values (im may be NULL) at `scale` into the
 * plaintext d_pt[level+1][N] (NTT domain).  Slot j sits at zeta^(5^j),
 * zeta = exp(i pi/N); coefficients are round-half-even(scale * t_k).
 * RBK_EINVAL if a coefficient reaches 2^62. */
int rbk_encode(rbk_ctx *ctx, const double *re, const double *im, size_t n, int level, double scale, uint64_t *d_pt);
/* Decode the first n slots of d_pt (NTT domain, level `level`) at `scale`
 * into host re[n] / im[n] (im may be NULL).  Uses the exact centred value
 * modulo q_0 q_1 (q_0 at level 0): the plaintext must satisfy
 * |m| < q_0 q_1 / 2.  Synchronises. */
int rbk_decode(rbk_ctx *ctx, const uint64_t *d_pt, int level, double scale, double *re, double *im, size_t n);
/* ct = (v pk0 + e0 + m, v pk1 + e1); v, e0, e1: host [N] small integers. */
int rbk_encrypt(rbk_ctx *ctx, const uint64_t *d_pt, int level, const int64_t *v, const int64_t *e0, const int64_t *e1,
                uint64_t *d_ct);
/* m = c0 + c1 s (NTT domain), d_pt[level+1][N]. */
int rbk_decrypt(rbk_ctx *ctx, const uint64_t *d_ct, int level, uint64_t *d_pt);

/* ---- slot-wise ring operations (Section 3, eqs. add / sub / mult) -------- */
/* npoly polynomials of level+1 limbs each (2 for a ciphertext). */
int rbk_add(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level, int npoly);
int rbk_sub(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level, int npoly);
int rbk_neg(rbk_ctx *ctx, const uint64_t *d_a, uint64_t *d_out, int level, int npoly);
/* pointwise product of npoly polynomials with as many polynomials */
int rbk_mul_poly(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level, int npoly);
/* ct (x) pt: both ciphertext polynomials times the plaintext d_pt[l+1][N] */
int rbk_mul_plain(rbk_ctx *ctx, const uint64_t *d_ct, const uint64_t *d_pt, uint64_t *d_out, int level);
/* ct (+) pt: the plaintext is added to c0 */
int rbk_add_plain(rbk_ctx *ctx, const uint64_t *d_ct, const uint64_t *d_pt, uint64_t *d_out, int level);
/* every limb i of npoly polynomials times the integer scal[i] (host, < q_i) */
int rbk_mul_scalar(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *scal, uint64_t *d_out, int level, int npoly);
/* ct + the constant polynomial with residues scal[i] (host, < q_i) */
int rbk_add_scalar(rbk_ctx *ctx, const uint64_t *d_ct, const uint64_t *scal, uint64_t *d_out, int level);
/* Scale-checked forms for callers that pass each operand's scale: the
 * slot-wise sum or difference (eqs. add / sub) is only the sum of the
 * messages when both operands carry the same scale, so these return
 * RBK_ESCALE unless |scale_a / scale_b - 1| < 2^-30 (RBK_EINVAL for a scale
 * that is not positive) and otherwise compute rbk_add / rbk_sub (one
 * ciphertext, npoly = 2) or rbk_add_plain, with *scale_out = scale_a
 * (scale_out may be NULL). */
int rbk_add_scaled(rbk_ctx *ctx, const uint64_t *d_a, double scale_a, const uint64_t *d_b, double scale_b,
                   uint64_t *d_out, int level, double *scale_out);
int rbk_sub_scaled(rbk_ctx *ctx, const uint64_t *d_a, double scale_a, const uint64_t *d_b, double scale_b,
                   uint64_t *d_out, int level, double *scale_out);
int rbk_add_plain_scaled(rbk_ctx *ctx, const uint64_t *d_ct, double scale_ct, const uint64_t *d_pt, double scale_pt,
                         uint64_t *d_out, int level, double *scale_out);
/* (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1); d_out[3][l+1][N] */
int rbk_tensor(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level);

/* ---- hybrid key switching ----------------------------------------------- */

/* ModUp: digits of alpha limbs of d_d[l+1][N], each extended by fast base
 * conversion to q_0..q_l, p_0..p_{n_p-1}: d_ext[beta_l][l+1+n_p][N]. */
int rbk_modup(rbk_ctx *ctx, const uint64_t *d_d, uint64_t *d_ext, int level);
/* (u0, u1) = sum_j ext_j (b_j, a_j) with the key of Galois element g
 * (g = 0: relinearisation key); d_u[2][l+1+n_p][N]. */
int rbk_key_inner_product(rbk_ctx *ctx, const uint64_t *d_ext, uint64_t g, uint64_t *d_u, int level);
/* ModDown of npoly polynomials d_u[npoly][l+1+n_p][N] -> d_out[npoly][l+1][N]:
 * (u_Q - BConv_{P->Q}(u_P)) * P^-1. */
int rbk_moddown(rbk_ctx *ctx, const uint64_t *d_u, uint64_t *d_out, int level, int npoly);
/* KS(d) = ModDown(<ModUp(d), key_g>), d_out[2][l+1][N] */
int rbk_keyswitch(rbk_ctx *ctx, uint64_t g, const uint64_t *d_d, uint64_t *d_out, int level);

/* ---- ciphertext operations ---------------------------------------------- */

/* Homomorphic product with relinearisation (eq. mult): (d0, d1) + KS(d2).
 * The scale of the result is the product of the scales. */
int rbk_mult_relin(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level);
/* Rescale by q_l: out_i = (c_i - centred(c_l)) q_l^-1 mod q_i; d_out[2][l][N].
 * Input and output must not overlap (their strides differ): RBK_EINVAL. */
int rbk_rescale(rbk_ctx *ctx, const uint64_t *d_ct, uint64_t *d_out, int level);
/* NTT-domain automorphism X -> X^g of npoly polynomials of level+1 limbs */
int rbk_automorph(rbk_ctx *ctx, const uint64_t *d_in, uint64_t *d_out, int level, int npoly, uint64_t g);
/* Rot(ct, k) of Section 3: slot j of the result is slot j+k (mod N/2) of ct.
 * Needs the Galois key of 5^k.  ENOKEY otherwise. */
int rbk_rotate(rbk_ctx *ctx, const uint64_t *d_ct, uint64_t *d_out, int level, int64_t k);
/* complex conjugation of every slot (Galois element 2N-1) */
int rbk_conjugate(rbk_ctx *ctx, const uint64_t *d_ct, uint64_t *d_out, int level);
/* Hoisted rotations (Halevi-Shoup 2018): one ModUp of c1 shared by n
 * rotations ks[n]; d_outs[n][2][l+1][N]. */
int rbk_rotate_hoisted(rbk_ctx *ctx, const uint64_t *d_ct, const int64_t *ks, int n, uint64_t *d_outs, int level);

/* ---- batched forms ------------------------------------------------------ */
/* The same results as `count` separate calls, from one set of launches: the
 * NTTs, base conversions and key inner products of all ciphertexts go into
 * single kernels, and each key word is read once per launch for the batch. */

/* d_a, d_b, d_out: [count][2][l+1][N] */
int rbk_mult_relin_batch(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out, int level, int count);
/* d_ct: [count][2][l+1][N] -> d_out: [count][2][l][N]; no overlap (RBK_EINVAL) */
int rbk_rescale_batch(rbk_ctx *ctx, const uint64_t *d_ct, uint64_t *d_out, int level, int count);
/* For callers that cannot allocate device memory (work recorded under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and residues as rbk_rescale_batch, with its scratch
 * (2 x count x (1 + level) x N words) taken from a fixed device array of
 * RBK_NOALLOC_SCRATCH_BYTES that each GPU holds from the first context
 * created on it until the process ends.  The call allocates nothing (no
 * hipMalloc / hipFree, no library allocation).  Errors: RBK_EINVAL when the
 * scratch would exceed the array (or d_ct and d_out overlap), RBK_ESTATE while
 * per-kernel timers are on.  All calls on one GPU share the array: calls whose
 * work overlaps in time on that GPU (other streams, other threads) race. */
#define RBK_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rbk_rescale_batch_noalloc(rbk_ctx *ctx, const uint64_t *d_ct, uint64_t *d_out, int level, int count);
/* d_ct: [count][2][l+1][N] -> d_outs: [count][n][2][l+1][N].  The
 * rotations' ModDowns run on the side streams set by rbk_set_lanes; the
 * call's work is complete, as for every call, once the context stream
 * reaches the point where it was issued. */
int rbk_rotate_hoisted_batch(rbk_ctx *ctx, const uint64_t *d_ct, const int64_t *ks, int n, uint64_t *d_outs, int level,
                             int count);
/* out = add + Rot(ct, k) for count ciphertexts: Section 3's Rot followed by
 * Add, in one pass where the ring allows (the rotation's ModDown adds `add`),
 * the step of the rotate-and-sum that the packed MLP's row and column sums
 * (Section 4.1) and the bootstrap's giant steps repeat.  d_ct, d_add, d_out:
 * [count][2][l+1][N], NTT domain.  d_add may be d_ct (ct + Rot(ct, k)) or
 * d_out (accumulation in place); d_ct must not overlap d_out, nor d_add
 * overlap d_out other than being it (RBK_EINVAL).  RBK_ENOKEY without the
 * Galois key of 5^k.  Residues equal rbk_rotate followed by rbk_add. */
int rbk_rotate_add_batch(rbk_ctx *ctx, const uint64_t *d_ct, const uint64_t *d_add, uint64_t *d_out, int level,
                         int count, int64_t k);

/* ---- descriptor lists: uneven level and ring degree per launch ---------- */
/* Work whose shapes differ goes through one set of launches: the transforms
 * run on a persistent grid that walks a list of descriptors, the other
 * kernels read a per-ciphertext level table.  Descriptors are packed on the
 * host and uploaded on the context stream, so list calls are refused
 * (RBK_ESTATE) during graph capture.  Ring degrees up to 2^16. */

/* one limb of one polynomial: N residues of ctx's ring at d_limb (device),
 * modulo prime index `prime` of ctx (Q primes, then special primes) */
typedef struct {
    const rbk_ctx *ctx;
    uint64_t *d_limb;
    int prime;
    int pad;
} rbk_ntt_item;
/* In-place forward (inverse = 0) or inverse NTT of every limb of the list,
 * each in its own context's ring (contexts on the device of ctx), launched
 * on ctx's stream.  The same results as per-context rbk_ntt calls (inputs
 * in [0, q), outputs in [0, q)); a limb must not appear twice in one list.
 * RBK_EUNSUPPORTED for a ring degree above 2^16. */
int rbk_ntt_list(rbk_ctx *ctx, const rbk_ntt_item *items, int n, int inverse);
/* out_i = rescale(mult_relin(a_i, b_i)) for count ciphertexts of ctx at the
 * uneven levels levels[i] (host array, 1 <= levels[i] <= L).  With Lm the
 * largest level: d_a, d_b: [count][2][Lm+1][N], ciphertext i in limbs
 * 0..levels[i] of its slot; d_out: [count][2][Lm][N], ciphertext i written
 * to limbs 0..levels[i]-1 (the rest of its slot is left as it was).  The
 * same residues as rbk_mult_relin_batch followed by rbk_rescale_batch at
 * each ciphertext's level.  d_out must not overlap d_a or d_b (RBK_EINVAL). */
int rbk_mult_relin_rescale_list(rbk_ctx *ctx, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out,
                                const int *levels, int count);

/* Ciphertexts of DIFFERENT contexts (ring degree, modulus chain, special
 * primes, relinearisation key; all on the device of ctx) in one set of
 * launches: item i computes d_out = Rescale(mult_relin(d_a, d_b)) in its own
 * context at its own level (1..L of that context), exactly as
 * rbk_mult_relin followed by rbk_rescale there (Section 3: mult, then the
 * switch to the next prime).  d_a, d_b: [2][level+1][N_i], d_out:
 * [2][level][N_i], NTT domain; an item's inputs and output must not overlap.
 * Runs on ctx's stream with ctx's workspace and descriptor arena; the item
 * contexts are only read (tables and keys) and must not be in use on another
 * thread.  Ring degrees 2^4..2^16 (the list transform), at most 16 primes per
 * digit, 16 special primes and 8 digits.  Not capturable (descriptors are
 * uploaded per call). */
typedef struct {
    rbk_ctx *ctx;
    const uint64_t *d_a;
    const uint64_t *d_b;
    uint64_t *d_out;
    int level;
    int pad;
} rbk_mr_item;
int rbk_mult_relin_rescale_multi(rbk_ctx *ctx, const rbk_mr_item *items, int n);

/* ---- approximate bootstrapping (Section 3: encoding step, scaled-sine
 *      modular reduction, decoding step; Cheon et al. 2018, Bossuat et al.
 *      2021) ------------------------------------------------------------- */

/* K         : bound on |I| after ModRaise; EvalMod interpolates on [-K-1, K+1]
 * degree    : degree of the Chebyshev interpolant of cos(2 pi (x - 1/4) / 2^r)
 * double_angle : r, the number of y <- 2y^2 - 1 steps
 * cts_levels, stc_levels : sparse transforms of CoeffToSlot and SlotToCoeff
 * log2_rho  : inputs are pre-scaled by a power of two to a scale in
 *             (D/2, D], D = 2^(bits(q_0) - log2_rho) */
typedef struct {
    uint32_t K;
    uint32_t degree;
    uint32_t double_angle;
    uint32_t cts_levels;
    uint32_t stc_levels;
    uint32_t log2_rho;
} rbk_boot_params;

/* Build the bootstrapping plan for the full chain of the context: levels,
 * scales, the encoded diagonals of the transforms (device encoder) and the
 * scalar constants of EvalMod.  ELEVEL if the chain is too short. */
int rbk_boot_setup(rbk_ctx *ctx, const rbk_boot_params *params);
/* Rotation indices (0 < k < N/2) whose Galois keys bootstrapping needs, in
 * increasing order; the conjugation key (2N-1) is needed as well.  Writes at
 * most max entries, returns the total count. */
int rbk_boot_rotations(const rbk_ctx *ctx, int64_t *ks, int max);
/* levels[4] = {top level L, EvalMod input level, SlotToCoeff input level,
 * output level}; counts of encoded diagonals and scalar constants. */
int rbk_boot_info(const rbk_ctx *ctx, int *levels, int *n_plain, int *n_scalar);
/* level of every diagonal / scalar constant, in plan order */
int rbk_boot_constant_levels(const rbk_ctx *ctx, int *plain_levels, int *scalar_levels);
/* Constants in plan order, coefficient domain: diagonal i is [level_i+1][N]
 * residues, scalar i is [level_i+1] residues, all concatenated.  Plan order:
 * CoeffToSlot transforms then SlotToCoeff transforms, each by giant step then
 * baby step; EvalMod scalars in evaluation order.  Either pointer may be NULL.
 * import replaces the plan's constants (residues must be below their prime). */
int rbk_boot_export(rbk_ctx *ctx, uint64_t *plains, uint64_t *scalars);
int rbk_boot_import(rbk_ctx *ctx, const uint64_t *plains, const uint64_t *scalars);
/* Bootstrap count level-0 ciphertexts d_in[count][2][1][N] at scales
 * scales_in[count] into d_out[count][2][out+1][N] (out = the output level).
 * scales_out receives the scale of each result.  Needs the relinearisation
 * key, the conjugation key and every key of rbk_boot_rotations. */
int rbk_bootstrap_batch(rbk_ctx *ctx, const uint64_t *d_in, const double *scales_in, uint64_t *d_out, double *scales_out,
                        int count);
int rbk_bootstrap(rbk_ctx *ctx, const uint64_t *d_in, double scale_in, uint64_t *d_out, double *scale_out);

/* ---- packed MLP training step (paper Section 4; Algorithms 1 and 2) ------ */

/* An MLP of H encrypted local-loss blocks packed into r x c slot matrices
 * (Section 4.1, r c = N/2, slot (i, j) at index i c + j).  Block h (1-based)
 * is an RE-block for odd h (RE-FC layer in the row-wise format, CE-FC local
 * classifier in the column-wise format) and a CE-block for even h.  Its
 * forward pass, RSS gradient, backward pass and NAG-style update follow
 * Algorithm 1 and Algorithm 2; the products are RE-Matmul / CE-Matmul
 * (SumRows / SumCols of Section 3).
 *
 *  k0        input width; wider than r means ceil(k0 / r) row tiles of the
 *            first layer (its input, weights, gradients and velocities are
 *            one ciphertext per tile, and RE-Matmul sums the tiles first)
 *  widths    k_1..k_H; odd layers k_h <= c, even layers k_h <= r, and the
 *            input of every layer but the first fits its side (r or c)
 *  n_out     o, the outputs of every local classifier (o <= r and o <= c)
 *  act       f(z) = act[0] z + act[1] z^2 + act[2] z^3; the leading non-zero
 *            coefficient (act[2], else act[1]) must be positive.  The paper's
 *            activation z + z^2 is {1, 1, 0}
 *  gamma, eta, mu   learning rate, decay rate, momentum of Algorithm 2
 *  log2_scale       the scale 2^log2_scale of the updated W and V
 *  flags     RBK_MLP_LITERAL_DERIV: dZ = 1 + 2 dA as printed in Section
 *            4.3.3 instead of the chain rule dZ = dA (.) f'(Z);
 *            RBK_MLP_L2_DECAY: decay dW + eta W instead of (1 + eta) dW
 *
 * The batch gradient is the mean over the b samples.  The update folds the
 * decay and the constants gamma, gamma mu, gamma mu^2 into one scalar per
 * operand: W' = W - c_w dW - c_wv V and V' = c_v dW + c_vv V, one level each.
 * Every ciphertext carries an exact float64 scale: a product of ciphertexts
 * has scale s_a s_b / q_l, a product with a constant c uses the integer
 * round(c q_l T / s) so that the rescaled result has the scale T it must
 * meet, the SumCols mask is encoded at scale q_l, and an affine map a x + b
 * (a > 0) of one ciphertext only changes its scale to s / a and adds
 * round(b s / a).  Additions then always meet equal scales (RBK_ESCALE
 * otherwise). */
#define RBK_MLP_LITERAL_DERIV 1u
#define RBK_MLP_L2_DECAY 2u

typedef struct rbk_mlp rbk_mlp;

typedef struct {
    uint32_t k0;
    uint32_t n_layers;
    const uint32_t *widths;
    uint32_t n_out;
    uint32_t r, c;
    double act[3];
    double gamma, eta, mu;
    double log2_scale;
    uint32_t flags;
} rbk_mlp_desc;

/* Validate the description against the context's N and create the step's
 * runner (device memory is taken on the first step and kept).  *out owned by
 * the caller; destroy it before its context (rbk_ctx_destroy returns
 * RBK_ESTATE while MLPs of the context are alive). */
int rbk_mlp_create(rbk_ctx *ctx, const rbk_mlp_desc *desc, rbk_mlp **out);
int rbk_mlp_destroy(rbk_mlp *mlp);
/* info[0] = input tiles, info[1] = state ciphertexts, info[2] = levels one
 * step consumes below the level of the weights (Table 1's depth) */
int rbk_mlp_info(const rbk_mlp *mlp, int *info);
/* rotation indices (both signs) the step needs Galois keys for; writes at
 * most max, returns the count */
int rbk_mlp_rotations(const rbk_mlp *mlp, int64_t *ks, int max);
/* The state is, per block h: the W tiles (one ciphertext each), W*, the V
 * tiles, V*.  set_state copies d_ct[2][level+1][N] (NTT domain) with its
 * scale into slot idx; get_state returns level and scale and, if d_ct is not
 * NULL, copies the ciphertext out.  V slots are not read at t = 1. */
int rbk_mlp_set_state(rbk_mlp *mlp, int idx, const uint64_t *d_ct, int level, double scale);
int rbk_mlp_get_state(rbk_mlp *mlp, int idx, uint64_t *d_ct, int *level, double *scale);
/* Float64 weights in and out of the encrypted state (Algorithm 1's W, W*
 * and the velocities V, V*).  Per block h (0-based index h-1): W[h-1] is
 * k_{h-1} x k_h and Wstar[h-1] is k_h x o, row-major; V / Vstar the same
 * shapes (either NULL: zero velocities / not read).  set packs each matrix
 * into its slot matrix (Section 4.1: RE-blocks hold W in the row-wise
 * format, tile t taking rows t r .. t r + r - 1, and W* column-wise;
 * CE-blocks the other way round), encodes it at `level` and scale
 * 2^log2_scale and encrypts it with randomness drawn from (seed, index =
 * state slot) (needs the public key), replacing the state.  get decrypts
 * (needs the secret key), decodes each state ciphertext at its own scale and
 * unpacks it; NULL arrays are skipped.  Both synchronise. */
int rbk_mlp_set_weights(rbk_mlp *mlp, const double *const *W, const double *const *Wstar, const double *const *V,
                        const double *const *Vstar, int level, uint64_t seed);
int rbk_mlp_get_weights(rbk_mlp *mlp, double *const *W, double *const *Wstar, double *const *V, double *const *Vstar);
/* Use d_pt[level+1][N] (NTT domain, encoded at scale q_level) as the SumCols
 * mask plaintext at `level` instead of the library's own encoding. */
int rbk_mlp_set_mask(rbk_mlp *mlp, int level, const uint64_t *d_pt);

/* One training step t >= 1 on b samples, all at `level` and `scale`:
 *   d_x     [b][tiles][2][level+1][N]  inputs in the expanded format
 *   d_y_exp [b][2][level+1][N]         one-hot labels, expanded format
 *   d_y_rep [b][2][level+1][N]         the same labels, repeated format
 * Afterwards every state ciphertext is bootstrapped (one batched call; the
 * context needs rbk_boot_setup and its keys) unless RBK_MLP_NO_BOOTSTRAP.
 * RBK_MLP_PER_SAMPLE runs the samples one at a time (the plain form; the
 * default processes the b samples of every operation in one launch set);
 * the residues are the same either way.  In that batched form block h's
 * classifier, loss and backward pass run on a second stream of the MLP,
 * beside block h+1's forward pass (Section 4.2.3: no information flows
 * between blocks in the backward pass), and the updates wait for both;
 * RBK_MLP_SEQUENTIAL keeps everything on the context stream, as do per-kernel
 * timers and graph capture.  The residues are the same either way.  Needs
 * the relinearisation key and the keys of rbk_mlp_rotations.  RBK_ELEVEL if
 * a product would go below level 0. */
#define RBK_MLP_NO_BOOTSTRAP 1u
#define RBK_MLP_PER_SAMPLE 2u
#define RBK_MLP_SEQUENTIAL 4u
int rbk_mlp_train_step(rbk_mlp *mlp, const uint64_t *d_x, const uint64_t *d_y_exp, const uint64_t *d_y_rep, int b,
                       int level, double scale, int t, uint32_t step_flags);
/* Encrypted inference with early exit (Section 4.2.3: after training, the
 * local classifiers can serve as exits): the forward pass of blocks
 * 1..last on b samples d_x [b][tiles][2][level+1][N] (expanded format, at
 * `level` and `scale`), and the output Yhat_h of every local classifier
 * h <= last.  d_out [last][b][2][level+1][N]: sample i's output of block h
 * is the ciphertext [2][levels[h-1]+1][N] at the start of slot (h-1, i),
 * scale scales[h-1] (levels / scales may be NULL).  A RE-block's output is
 * in the expanded format (class j in row j), a CE-block's in the repeated
 * format (class j in column j).  Needs the W and W* state of blocks
 * 1..last, the relinearisation key and the keys of rbk_mlp_rotations;
 * deeper blocks are not evaluated.  Synchronises. */
int rbk_mlp_infer(rbk_mlp *mlp, const uint64_t *d_x, int b, int level, double scale, int last, uint64_t *d_out,
                  int *levels, double *scales);
/* The integer constants the last step multiplied or added, in evaluation
 * order (with RBK_MLP_PER_SAMPLE: sample by sample, block by block, then
 * the updates).  Writes at most max, returns the count. */
int rbk_mlp_scalars(const rbk_mlp *mlp, int64_t *out, int max);

/* ---- serving loop ---------------------------------------------------------- */

/* Encrypted-training jobs of several tenants on one GPU.  A tenant is a
 * context with its keys (and bootstrap plan) set up; from rbk_server_add_tenant
 * until rbk_server_destroy the server owns it: it gets a stream of its own and
 * a worker thread of its own, runs on one lane (rbk_set_lanes; restored at
 * destroy; training steps with RBK_MLP_SEQUENTIAL), and the caller must not
 * call into it (the device memory a job
 * names stays the caller's).  Work of different tenants overlaps on the
 * device.
 *
 * Admission: an HBM ledger starts with every tenant's resident bytes (its
 * evaluation keys and bootstrap diagonals); a job is admitted, in arrival
 * order, once its footprint fits the budget next to the ledger (later jobs
 * may pass a job that does not fit, at most 8 times in a row).  Footprints
 * are working-set estimates, with n = min(count, chunk cap): mult
 * count + 5.5 n ciphertexts + key-switch workspace of n; bootstrap n x 48
 * top-level ciphertexts; training step b x 24 ciphertexts + workspace.
 *
 * Batching: whenever a tenant's stream is free, its oldest admitted job runs
 * together with every later admitted job of the same kind and level, up to
 * max_batch ciphertexts (max_boot_batch for bootstraps; training steps run
 * alone).  A batch runs in chunks of at most that many ciphertexts, which
 * bounds each tenant's workspace.  Results do not depend on the batching:
 * the batched operations are the per-ciphertext ones. */
#define RBK_JOB_MULT_RESCALE 1  /* out = Rescale(mult_relin(a_i, b_i)), i < count */
#define RBK_JOB_BOOTSTRAP 2     /* out_i = Bootstrap(a_i) (level-0 part of a_i) */
#define RBK_JOB_TRAIN_STEP 3    /* `count` steps t0, t0+1, ... of an MLP */

typedef struct rbk_server rbk_server;

typedef struct {
    int kind;
    int tenant;
    int count;            /* ciphertexts (mult, bootstrap) or steps (train) */
    int level;            /* mult: operation level l >= 1; train: level of x and y */
    int in_level;         /* layout level of d_a / d_b: [count][2][in_level+1][N], in_level >= level */
    const uint64_t *d_a;  /* mult, bootstrap inputs (NTT domain) */
    const uint64_t *d_b;  /* mult second inputs */
    uint64_t *d_out;      /* mult: [count][2][l][N]; bootstrap: [count][2][out+1][N] */
    const double *scales_in;  /* bootstrap: host [count], copied at submission */
    double *scales_out;       /* bootstrap: host [count], written before the job completes (may be NULL) */
    rbk_mlp *mlp;             /* train: an MLP of this tenant's context */
    const uint64_t *d_x, *d_y_exp, *d_y_rep;  /* train: as rbk_mlp_train_step */
    int b;
    double scale;
    int t0;
} rbk_job;

typedef struct {
    int status;         /* 0 or the job's RBK_E* code */
    double latency_ms;  /* submission to completion */
    double queue_ms;    /* submission to start on the device */
    double run_ms;      /* start to completion of its batch */
    int batch_cts;      /* ciphertexts (or 1 step) in the batch it ran in */
} rbk_job_result;

/* budget: HBM bytes the ledger may hold; max_batch / max_boot_batch:
 * ciphertexts per launch of mult+rescale / bootstrap work */
int rbk_server_create(uint64_t hbm_budget, int max_batch, int max_boot_batch, rbk_server **out);
/* RBK_ENOMEM if the tenant's resident bytes do not fit; before rbk_server_start */
int rbk_server_add_tenant(rbk_server *srv, rbk_ctx *ctx, int *tenant);
int rbk_server_start(rbk_server *srv);
/* Thread-safe; returns at once with the job's id.  RBK_ENOMEM if the job can
 * never fit the budget.  Inputs must be ready on the device (the caller's
 * stream synchronised) and stay valid until the job completes. */
int rbk_server_submit(rbk_server *srv, const rbk_job *job, uint64_t *id);
/* Block until job id completes, fill *res and forget the job.  Returns the
 * job's status (its message through rbk_last_error). */
int rbk_server_wait(rbk_server *srv, uint64_t id, rbk_job_result *res);
/* Block until every submitted job has completed. */
int rbk_server_drain(rbk_server *srv);
/* stats[6] = {jobs completed, batches run, jobs that ran merged with others,
 * peak ledger bytes, ledger bytes now, budget} */
int rbk_server_stats(rbk_server *srv, uint64_t *stats);
/* Cross-tenant batching (off by default; set before rbk_server_start): a
 * tenant's mult batch also takes admitted mult jobs of other tenants whose
 * contexts have special primes and a ring degree up to 2^16 (any level, any
 * ring degree, oldest first, within max_batch), and runs them in one
 * multi-context launch set (rbk_mult_relin_rescale_multi: every ciphertext
 * with its own tenant's keys and tables) on the leading tenant's stream.
 * The other contexts are only read; their ModUp tables of every level are
 * built at rbk_server_start. */
int rbk_server_set_cross_tenant(rbk_server *srv, int on);
/* *n = jobs that ran in a batch led by another tenant's worker */
int rbk_server_cross_merged(rbk_server *srv, uint64_t *n);
/* Run what was submitted, stop the workers, give the contexts their streams
 * back, free the server. */
int rbk_server_destroy(rbk_server *srv);

/* ---- autotuner -------------------------------------------------------------- */

/* Launch parameters that change speed but never a residue (cfg: int[3]):
 *   cfg[0] = logC, the NTT split (a limb is a 2^(logN-logC) x 2^logC matrix;
 *            for 13 <= logN <= 16 both sides must be 2^6 .. 2^8, for
 *            logN = 17 logC is 8 or 9);
 *   cfg[1] = ciphertexts per thread of the fused key inner products (1..64);
 *   cfg[2] = NTT chunk: limbs covered by one pair of pass launches before
 *            the next chunk (>= 0; 0 = the whole batch at once).
 * rbk_autotune times every candidate on the batched key-switching shape
 * (level, count) with HIP events on the context stream and keeps the
 * fastest.  With cache_path (a text file) it first looks up the GPU
 * architecture and shape there and appends what it measured.  cfg (may be
 * NULL) receives the configuration in force. */
int rbk_autotune(rbk_ctx *ctx, int level, int count, const char *cache_path, int *cfg);
int rbk_tune_get(const rbk_ctx *ctx, int *cfg);
int rbk_tune_set(rbk_ctx *ctx, const int *cfg);

/* ---- graph capture ---------------------------------------------------------- */

/* Record the device work of a sequence of calls on the context's stream into
 * a HIP graph and replay it with one launch.  Between rbk_capture_begin and
 * rbk_capture_end nothing executes: the calls enqueue their kernels and
 * copies into the graph (host-side results such as bootstrap output scales
 * are those computed while capturing).  Requirements:
 *  - the context is on a stream other than the default one (rbk_set_stream);
 *  - the same sequence ran once before, so that every workspace, register
 *    pool and mask is already sized: a call that would grow one fails with
 *    RBK_ESTATE instead (the capture must then be ended and discarded);
 *  - calls that transfer host data or synchronise (keygen, encode, decode,
 *    encrypt, bootstrap setup/import/export, timers, set_state) are refused;
 *  - the graph reads and writes the device addresses named while capturing:
 *    replays recompute from whatever those buffers hold at launch time
 *    (an MLP's state buffers keep their addresses across steps, so replaying
 *    a captured step t >= 2 runs the following steps).
 * No memset node is recorded (buffers are cleared by kernels). */
typedef struct rbk_graph rbk_graph;
int rbk_capture_begin(rbk_ctx *ctx);
int rbk_capture_end(rbk_ctx *ctx, rbk_graph **out);
/* enqueue the captured work on the context's current stream */
int rbk_graph_launch(rbk_graph *graph);
int rbk_graph_destroy(rbk_graph *graph);

/* ---- lanes --------------------------------------------------------------- */
/* A batch of hoisted rotations (rbk_rotate_hoisted_batch) runs the
 * independent ModDowns of its rotations round-robin on n side streams (lanes,
 * default priority) that join the context stream before the call returns;
 * each lane has tp/conv scratch of its own in the workspace (batches of up to
 * 4 ciphertexts instead run the ModDowns of all rotations as one set of
 * launches).  The bootstrap
 * runs the giant steps of its linear transforms on the same lanes (each with
 * a key-switching workspace and registers of its own; partial sums added on
 * the context stream) and, for batches of up to 4 ciphertexts, the EvalMod
 * products of one dependency depth.  Lanes overlap one rotation's arithmetic-bound kernels
 * with another's memory-bound ones, and small kernels of single-ciphertext
 * calls with each other; the default is 3; n = 1 runs everything on the
 * context stream (kernels do not overlap, so profiler durations are each
 * kernel's own).  Residues do not depend on n.  Lanes are not used while
 * timers run or while the stream is captured (a captured graph is one chain
 * of kernels).  n outside 1..3: RBK_EINVAL, setting unchanged. */
int rbk_set_lanes(rbk_ctx *ctx, int n);

/* ---- per-kernel timers -------------------------------------------------- */
/* With timers on, every kernel launch on the context stream is bracketed by
 * HIP events.  Class `cls` = 0, 1, ... names one kernel (rbk_timer_name);
 * rbk_timer_read returns its summed duration in ms, its number of launches,
 * and the algorithmic HBM bytes of those launches (the data each launch must
 * read and write, e.g. one read and one write of every limb for an NTT pass).
 * Both synchronise the stream. */
int rbk_timer_enable(rbk_ctx *ctx, int on);   /* resets all timers and the key-switch count */
int rbk_timer_read(rbk_ctx *ctx, int cls, double *ms, uint64_t *launches, double *bytes);
/* kernel name of class cls, NULL past the last class */
const char *rbk_timer_name(int cls);
/* Key switches issued since the last rbk_timer_enable (each switched
 * polynomial of a relinearisation or rotation counts one) and their method
 * bytes, the least HBM traffic the operation needs: per key switch at level
 * l, 2 (l+1) N words (the switched polynomial read, one polynomial written),
 * plus beta_l x 2 x (l+1+n_p) x N key words once per call (a batch shares
 * them); 8 bytes a word. */
int rbk_ks_stats(const rbk_ctx *ctx, uint64_t *n_keyswitch, double *method_bytes);

#ifdef __cplusplus
}
#endif
#endif
