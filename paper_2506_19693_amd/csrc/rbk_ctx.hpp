// Host-side context of librbk: parameters, prime tables, device constant
// tables, key material and the device workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <cstring>
#include <vector>

#include "rbk_internal.hpp"

// ModUp base-conversion tables of one level: digit j converts its own
// primes D_j = [lo_j, hi_j) to every other position of the extended basis.
struct ModUpTables {
    int level = -1;
    int beta = 0;
    std::vector<int> lo, n_in;
    u64 *d_A = nullptr;    // [beta][alpha]   (D_j / q_i)^-1 mod q_i
    u64 *d_Ash = nullptr;  // [beta][alpha]   Shoup quotients
    u64 *d_M = nullptr;    // [beta][alpha][E] (D_j / q_i) mod t * 2^64 mod t, by output position
};

// Per-kernel timers (HIP events around every launch of a kernel on the
// context stream), enabled by rbk_timer_enable.  'bytes' accumulates the
// algorithmic HBM bytes of each launch: what the kernel must read and write.
// Side-stream lanes (default priority) of a batch of hoisted rotations'
// ModDowns and of the bootstrap's giant steps: they overlap one rotation's
// VALU-bound kernels with another's memory-bound ones, and kernels too small
// to fill the GPU (single-ciphertext calls) with each other
#define RBK_LANES 3

enum KClass {
    KC_NTT_COLS_FWD = 0,
    KC_NTT_ROWS_FWD,
    KC_NTT_ROWS_INV,
    KC_NTT_COLS_INV,
    KC_BCONV_UP,
    KC_BCONV_DOWN,
    KC_IP,
    KC_MODDOWN_FIN,
    KC_TENSOR,
    KC_RESCALE,
    KC_ELEMENTWISE,
    KC_IP_P,
    KC_MODDOWN_IP,
    KC_NTT_ROWS_MD,
    KC_NTT_ROWS_IP,
    KC_COUNT
};

struct KTimer {
    std::vector<hipEvent_t> pending;  // begin/end pairs not yet read
    double ms = 0, bytes = 0;
    unsigned long launches = 0;
};

struct rbk_ctx_impl {
    int device = 0;
    hipStream_t stream = nullptr;
    int logN = 0;
    size_t N = 0;
    int nQ = 0, nP = 0, nT = 0, alpha = 1, beta = 1;
    int ntt_logC = 0;   // NTT split: a limb is a 2^(logN - ntt_logC) x 2^ntt_logC matrix
    int ip_cpc = 8;     // ciphertexts per thread of the fused key inner products
    // limbs per chunk of a two-pass NTT launch: both passes run over one chunk
    // before the next, so the intermediate can stay in the memory-side cache
    // (0: one pair of launches over the whole batch)
    int ntt_chunk = 512;
    int lanes = RBK_LANES;  // ModDown lanes of a batch of hoisted rotations (rbk_set_lanes)
    std::vector<u64> mod, psi;
    std::vector<PrimeC> h_pc;

    // device constant tables
    PrimeC *d_pc = nullptr;
    u64 *d_tw = nullptr, *d_tw_sh = nullptr, *d_itw = nullptr, *d_itw_sh = nullptr;
    u64 *d_last = nullptr, *d_last_sh = nullptr;
    double2 *d_twf = nullptr, *d_itwf = nullptr;
    FpC *d_fc = nullptr;
    NttTables *d_tabs = nullptr;  // device copy of tabs, for descriptor-list transforms
    NttTables tabs{};

    // ModDown P -> Q (level independent, indexed by Q prime)
    u64 *d_md_A = nullptr, *d_md_Ash = nullptr;  // [nP]
    u64 *d_md_M = nullptr;                       // [nP][nQ]   Montgomery form
    u64 *d_Pinv = nullptr, *d_Pinv_sh = nullptr; // [nQ]
    std::vector<u64> h_Pmod;                     // P mod q_i, every prime of Q
    u64 *d_Pmod = nullptr, *d_Pmod_sh = nullptr; // [nQ]
    int *d_pow5 = nullptr;                       // [N/2]  (5^j mod 2N - 1) / 2
    u64 *d_q0mod = nullptr;                      // [nQ]  q_0 mod q_i
    u64 *d_iq = nullptr, *d_iq_sh = nullptr;     // [nQ]  psi_i^(N/2), a square root of -1 mod q_i

    // rescale by q_l: [l][i] = q_l^-1 mod q_i, its Shoup quotient, q_l mod q_i
    u64 *d_rs_inv = nullptr, *d_rs_inv_sh = nullptr, *d_rs_qmod = nullptr;  // [nQ][nQ]

    std::map<int, ModUpTables> modup;

    // key material (NTT domain)
    u64 *d_s = nullptr;   // [nT][N] secret
    u64 *d_pk = nullptr;  // [2][nQ][N]
    DevKey relin;
    std::map<u64, DevKey> gal;

    // workspace (grow-only), or a caller's buffer (ws_ext, never grown or freed)
    u64 *ws = nullptr;
    size_t ws_words = 0;
    u64 *ws_ext = nullptr;

    std::vector<void *> owned;  // device allocations freed at destroy

    struct BootPlan *boot = nullptr;   // bootstrapping plan (boot.hip)
    int live_mlps = 0;                 // rbk_mlp objects built on this context (mlp.hip)

    bool timing = false;
    // the stream is being captured into a graph: nothing may grow, free or wait
    bool capturing = false;
    // graphs recorded on this context reference its workspaces: while any is
    // alive, a buffer that is replaced is retired instead of freed
    int live_graphs = 0;
    std::vector<void *> retired;
    hipError_t free_error = hipSuccess;  // first failed hipFree, reported at destroy
    // descriptor uploads of the list entry points: one device arena reused by
    // every call (stream order protects it) and two pinned host arenas used
    // in turn, each reusable once the event after its last copy has passed
    void *desc_dev = nullptr;
    size_t desc_dev_bytes = 0;
    void *desc_host[2] = {nullptr, nullptr};
    size_t desc_host_bytes[2] = {0, 0};
    hipEvent_t desc_evt[2] = {nullptr, nullptr};
    int desc_turn = 0;
    // side streams of the multi-lane ModDown of hoisted rotations (lazily
    // created); side_ev[RBK_LANES] forks the lanes off the context stream
    hipStream_t side[RBK_LANES] = {};
    hipEvent_t side_ev[RBK_LANES + 1] = {};
    mutable KTimer timers[KC_COUNT];
    // key switches since the last rbk_timer_enable and their method bytes:
    // per key switch at level l the switched polynomial is read and one
    // polynomial written (2 (l+1) N words), plus the key words of that level
    // (beta_l x 2 x (l+1+k) x N) once per call, shared by the call's batch
    unsigned long ks_units = 0;
    double ks_bytes = 0;
    mutable std::vector<hipEvent_t> event_pool;
};

// the opaque handle of the C ABI
struct rbk_ctx : rbk_ctx_impl {};

// Host-side packing of the descriptor arrays of one list call; every part is
// 16-byte aligned.  desc_upload copies the blob to the context's device
// arena on its stream and returns the device address (null on failure, with
// the error set and its code in *rc).
struct DescBlob {
    std::vector<char> h;
    template <class T>
    size_t put(const T *p, size_t n)
    {
        const size_t off = (h.size() + 15) & ~(size_t)15;
        h.resize(off + n * sizeof(T));
        if (n) std::memcpy(h.data() + off, p, n * sizeof(T));
        return off;
    }
};
char *desc_upload(rbk_ctx_impl *c, const DescBlob &b, int *rc);

// timer hooks around a launch (no-ops unless timing is enabled)
void kt_begin(const rbk_ctx_impl *c, int cls, hipStream_t st);
void kt_end(const rbk_ctx_impl *c, int cls, double bytes, hipStream_t st);

// ---- helpers implemented in api.hip ----
// count `count` key switches at `level` (one call, the key read once) for rbk_ks_stats
void ks_account(rbk_ctx_impl *c, const int *levels, int count, int key_level);
u64 *ws_reserve(rbk_ctx_impl *c, size_t words);
// the context's side streams and their fork / join events (created once)
int side_streams(rbk_ctx_impl *c);
// free a replaced device buffer, or keep it until the last graph is destroyed
void release_buffer(rbk_ctx_impl *c, void *p);
void dev_free(rbk_ctx_impl *c, void *p);
const ModUpTables &modup_tables(rbk_ctx_impl *c, int level);

// ---- kernel launchers implemented in kernels.hip ----
enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_NEG = 2, EW_MUL = 3, EW_COPY = 4, EW_ZERO = 5 };

struct ScalArg {
    u64 w[RBK_MAX_PRIMES];
    u64 wsh[RBK_MAX_PRIMES];
};

void ew_launch(const rbk_ctx_impl *c, EwOp op, const u64 *a, const u64 *b, u64 *out, int npoly, int nlimbs, LimbMap map,
               hipStream_t st);
void mul_scalar_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int npoly, int nlimbs, LimbMap map, const ScalArg &s,
                       hipStream_t st);
void add_scalar_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int nlimbs, const ScalArg &s, hipStream_t st);
void signed_to_limbs_launch(const rbk_ctx_impl *c, const i64 *v, u64 *out, int npoly, int nlimbs, LimbMap map,
                            hipStream_t st);
void tensor_launch(const rbk_ctx_impl *c, const u64 *a, const u64 *b, u64 *out, int level, int count, hipStream_t st);
void automorph_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int npoly, int nlimbs, u64 g, hipStream_t st);
void automorph_polys_launch(const rbk_ctx_impl *c, const u64 *in, long in_stride, u64 *out, long out_stride, int npoly,
                            int nlimbs, u64 g, hipStream_t st);
void bconv_modup_launch(const rbk_ctx_impl *c, const u64 *coef, long coef_stride, const u64 *own, long own_stride,
                        u64 *ext, long ext_stride, int level, int count, hipStream_t st);
void bconv_moddown_launch(const rbk_ctx_impl *c, const u64 *pcoef, long p_stride, u64 *conv, long conv_stride, int level,
                          int count, hipStream_t st);
void ip_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *u, long u_stride, int level,
               int count, u64 g, hipStream_t st);
void moddown_finish_launch(const rbk_ctx_impl *c, const u64 *u, long u_stride, const u64 *conv, long conv_stride,
                           const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level,
                           int count, hipStream_t st);
void ip_p_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *tp, int level, int count,
                 u64 g, hipStream_t st);
void moddown_ip_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, const u64 *conv,
                       long conv_stride, const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out,
                       long out_stride, int level, int count, u64 g, hipStream_t st);
// Inverse NTT of npoly x nlimbs limbs read from src (limb i of polynomial p
// at src + p src_stride + i N) into dst (same layout with dst_stride); src is
// left unchanged.
hipError_t ntt_inverse_from_launch(const rbk_ctx_impl *c, const u64 *src, long src_stride, u64 *dst, long dst_stride,
                                   int npoly, int nlimbs, LimbMap map, hipStream_t st);
// Rescale tail for the register NTT geometries: lifted ([npoly][level] limbs)
// = NTT of the centred lift of last ([npoly] limbs, coefficient domain), then
// out ([npoly][level]) = (in ([npoly][level+1]) - lifted) q_level^-1, the
// lift computed inside the column pass and the finish inside the row pass.
// Returns false (nothing launched) for other geometries.
bool rescale_fused_launch(const rbk_ctx_impl *c, const u64 *last, u64 *lifted, const u64 *in, u64 *out, int level,
                          int npoly, hipStream_t st);
// ModDown head: tp ([count][2][k] limbs) = the special-prime part of the key
// inner product, brought to the coefficient domain; for the register NTT
// geometries the inner product is computed inside the first iNTT pass.
void moddown_head_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *tp, int level,
                         int count, u64 g, hipStream_t st);
// ModDown tail: NTT of the converted special-prime part conv ([count][2][l+1]
// limbs) and the epilogue of moddown_ip_launch; for the register NTT
// geometries the row pass and the epilogue are one kernel.  conv is clobbered.
// Several key switches of one batch in one launch set (the rotations of a
// hoisted batch): per item a switching key, the Galois element its digits
// are read through, that of its addend, and the offset (words) of its
// outputs.  tp / conv hold item i's ciphertexts at slots i count ..
// i count + count - 1.  For the register NTT geometries only
// (moddown_items_ok).
#define KS_MAX_ITEMS 32
struct KsItems {
    const u64 *key[KS_MAX_ITEMS];
    u64 g[KS_MAX_ITEMS];
    u64 add_g[KS_MAX_ITEMS];
    long out_off[KS_MAX_ITEMS];
    int n;
};
bool moddown_items_ok(const rbk_ctx_impl *c);
void moddown_head_items_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *tp,
                               int level, int count, hipStream_t st);
// add2 (optional, the register geometries with special primes only:
// moddown_add2_ok): a second addend on both polynomials, read in place, with
// the rotation form of add (c0 only); it may be out itself
void moddown_tail_items_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const KsItems &I, u64 *conv,
                               const u64 *add, long add_stride, int add_both, u64 *out, long out_stride, int level,
                               int count, hipStream_t st, const u64 *add2 = nullptr, long add2_stride = 0);
void moddown_tail_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, const u64 *key, u64 *conv,
                         const u64 *add, long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level,
                         int count, u64 g, hipStream_t st, const u64 *add2 = nullptr, long add2_stride = 0);
bool moddown_add2_ok(const rbk_ctx_impl *c);
void rescale_lift_launch(const rbk_ctx_impl *c, const u64 *last, u64 *lifted, int level, int npoly, hipStream_t st);
void rescale_finish_launch(const rbk_ctx_impl *c, const u64 *in, const u64 *lifted, u64 *out, int level, int npoly,
                           hipStream_t st);
void keygen_launch(const rbk_ctx_impl *c, const u64 *a_ntt, const u64 *e_ntt, const u64 *s_from, u64 *key_out,
                   hipStream_t st);
void to_mont_launch(const rbk_ctx_impl *c, u64 *data, int npoly, int nlimbs, LimbMap map, bool inverse, hipStream_t st);
void encrypt_launch(const rbk_ctx_impl *c, const u64 *pt, const u64 *v, const u64 *e0, const u64 *e1, u64 *ct, int level,
                    hipStream_t st);
void encode_launch(const rbk_ctx_impl *c, const double *d_re, const double *d_im, size_t n, int level, double scale,
                   u64 *pt, double *fft_ws, int *err_flag, hipStream_t st);
void decode_launch(const rbk_ctx_impl *c, const u64 *pt_coef, int level, double scale, double *d_re, double *d_im,
                   size_t n, double *fft_ws, hipStream_t st);
void decrypt_launch(const rbk_ctx_impl *c, const u64 *ct, u64 *pt, int level, hipStream_t st);
void modraise_lift_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int level, int npoly, hipStream_t st);
void monomial_half_launch(const rbk_ctx_impl *c, const u64 *in, u64 *out, int npoly, int level, int neg, hipStream_t st);
// up to GT_MAX_G giant steps of one BSGS product over GT_MAX_B baby-step
// slots: out_j[c] = sum_b src_b[c] (.) pt_{j,b} (+ out_j[c] when add_j), count
// ciphertexts at level l (pt_{j,b} null: no term; outs distinct from srcs)
constexpr int GT_MAX_G = 4, GT_MAX_B = 8;
struct GiantTerms {
    const u64 *src[GT_MAX_B];  // baby slot b of ciphertext c at src[b] + c * stride[b]
    long stride[GT_MAX_B];
    u64 *out[GT_MAX_G];        // [count][2][l+1][N]
    const u64 *pt[GT_MAX_G][GT_MAX_B];
    int add[GT_MAX_G];
    int nb, ng;
};
void mac_giants_launch(const rbk_ctx_impl *c, const GiantTerms &T, int level, int count, hipStream_t st);
void add_scalar_batch_launch(const rbk_ctx_impl *c, const u64 *a, u64 *out, int level, int count, const ScalArg &s,
                             hipStream_t st);
void boot_free(rbk_ctx_impl *c);
size_t boot_resident_bytes(const rbk_ctx_impl *c);

// ---- pieces of api.hip shared with the bootstrap and MLP runners ----
// workspace words of the key-switching pipeline for `count` ciphertexts at level l
size_t ks_words(const rbk_ctx *c, int level, int count);
// KS of count polynomials d (d_stride apart) with `key`: out = KS(d) + add
// (add_both: both polynomials of add, else c0 only; perm_g: automorphism of
// the digits first, 0 for none); base: ks_words() of workspace
// (add2: a second addend on both polynomials, with the rotation form of add;
// moddown_add2_ok only; it may be out itself)
int keyswitch_run(rbk_ctx *c, const DevKey *key, u64 perm_g, const u64 *d, long d_stride, const u64 *add,
                  long add_stride, u64 add_g, int add_both, u64 *out, long out_stride, int level, int count, u64 *base,
                  const u64 *add2 = nullptr, long add2_stride = 0);
// out = Rot_g of count contiguous ciphertexts [count][2][l+1][N] (in and out
// must not overlap)
int rotate_batch_g(rbk_ctx *c, const u64 *in, u64 *out, int level, int count, u64 g);
// out = add2 + Rot_g(in), same layout; add2 may be out itself or in
int rotate_add_batch_g(rbk_ctx *c, const u64 *in, const u64 *add2, u64 *out, int level, int count, u64 g);
int rbk_set_error(int code, const char *msg);
// true when [a, a + a_words) and [b, b + b_words) share a word
bool ranges_overlap(const u64 *a, size_t a_words, const u64 *b, size_t b_words);
// rescale pieces: workspace words, argument checks, and the launches on a
// given workspace of rescale_ws_words() words
size_t rescale_ws_words(const rbk_ctx *c, int level, int count);
int rescale_check(rbk_ctx *c, const u64 *ct, u64 *out, int level, int count);
int rescale_run(rbk_ctx *c, const u64 *ct, u64 *out, int level, int count, u64 *ws);
// allocation-free entry points: looks up the device's scratch array (once per
// device, with that device current)
int noalloc_setup(int device);

// ---- seeded sampling (sample.hip) ----
// nonce purposes of the keystream (the quantity a block belongs to)
enum : u32 {
    RBK_SAMPLE_SECRET = 1,
    RBK_SAMPLE_PK_A = 2,
    RBK_SAMPLE_PK_E = 3,
    RBK_SAMPLE_KEY_A = 4,
    RBK_SAMPLE_KEY_E = 5,
    RBK_SAMPLE_ENC_V = 6,
    RBK_SAMPLE_ENC_E0 = 7,
    RBK_SAMPLE_ENC_E1 = 8,
};
// out [nlimbs][N]: limb t uniform modulo prime t of the context's table
void sample_uniform_launch(const rbk_ctx_impl *c, u64 *out, int nlimbs, u64 seed, u32 purpose, u32 id, u32 sub_hi,
                           hipStream_t st);
// out [N]: uniform ternary (gaussian = 0) or the sigma = 3.2 discrete Gaussian (gaussian = 1)
void sample_small_launch(const rbk_ctx_impl *c, i64 *out, u64 seed, u32 purpose, u32 id, u32 sub, int gaussian,
                         hipStream_t st);
// host: exactly h non-zero coefficients in {-1, +1}
void sample_ternary_hw_host(u64 seed, int logN, int h, i64 *out);
// *flag |= 1 when some residue of npoly x nlimbs limbs (prime i = limb i) is not below its prime
void check_residues_launch(const rbk_ctx_impl *c, const u64 *data, int npoly, int nlimbs, int *flag, hipStream_t st);

// ---- batches of uneven level (kernels.hip, list.hip) ----
// Per-ciphertext entry of a batch whose ciphertexts differ in level: the
// level and the ModUp tables of that level.
struct ListCt {
    int level;
    int pad;
    const u64 *A, *Ash, *M;
};
void tensor_list_launch(const rbk_ctx_impl *c, const u64 *a, const u64 *b, u64 *out, int Lm, int count,
                        const ListCt *cts, hipStream_t st);
void bconv_up_list_launch(const rbk_ctx_impl *c, const u64 *coef, long coef_stride, const u64 *d, long d_stride, u64 *ext,
                          long ext_stride, long dig_stride, int Lm, int count, const ListCt *cts, hipStream_t st);
void bconv_down_list_launch(const rbk_ctx_impl *c, const u64 *tp, u64 *conv, long conv_stride, int Lm, int count,
                            const ListCt *cts, hipStream_t st);
void ip_p_list_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, long dig_stride, const u64 *key, u64 *tp,
                      int Lm, int count, const ListCt *cts, hipStream_t st);
void moddown_ip_list_launch(const rbk_ctx_impl *c, const u64 *ext, long ext_stride, long dig_stride, const u64 *key,
                            const u64 *conv, long conv_stride, long per, const u64 *add, long add_stride, u64 *out,
                            long out_stride, int Lm, int count, const ListCt *cts, hipStream_t st);
// step 0: gather the last limbs; 1: lift; 2: finish
void rescale_list_launch(const rbk_ctx_impl *c, int step, const u64 *in, long in_poly_stride, u64 *last, u64 *lifted,
                         u64 *out, long out_poly_stride, int Lm, int count, const ListCt *cts, hipStream_t st);
