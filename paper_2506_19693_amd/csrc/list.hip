// Descriptor-list entry points: work of uneven level and ring degree in one
// set of launches.
//
//  * rbk_ntt_list: one limb per descriptor, each with its own context (ring
//    degree, prime tables), transformed by a persistent grid that walks the
//    (descriptor, tile) units of the whole list.
//  * rbk_mult_relin_rescale_list: ciphertexts of one context at uneven levels,
//    multiplied, relinearised (hybrid key switching) and rescaled together;
//    every NTT of the pipeline is a descriptor-list transform over exactly
//    the limbs each ciphertext owns, the other kernels take a per-ciphertext
//    level table.
//
// Descriptors are packed on the host once per call and uploaded to the
// context's descriptor arena; list calls are therefore not capturable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

namespace {

bool list_ntt_ok(int logN, int logC)
{
    if (logN <= 12) return logN >= 1;
    const int r = logN - logC;
    return logN <= 16 && r >= 6 && r <= 8 && logC >= 6 && logC <= 8;
}

// offsets of one packed descriptor-list transform inside a blob
struct PackedList {
    size_t items = 0, p1 = 0, p2 = 0;
    int n = 0, t1 = 0, t2 = 0;
};

PackedList pack_list(DescBlob &b, const std::vector<NttItem> &items)
{
    PackedList L;
    L.n = (int)items.size();
    std::vector<int> p1(items.size() + 1, 0), p2(items.size() + 1, 0);
    for (size_t i = 0; i < items.size(); i++) {
        p1[i + 1] = p1[i] + ntt_item_units(items[i].logN, true);
        p2[i + 1] = p2[i] + ntt_item_units(items[i].logN, false);
    }
    L.t1 = p1.back();
    L.t2 = p2.back();
    L.items = b.put(items.data(), items.size());
    L.p1 = b.put(p1.data(), p1.size());
    L.p2 = b.put(p2.data(), p2.size());
    return L;
}

void run_list(const char *dev, const PackedList &L, bool inverse, hipStream_t st)
{
    if (L.n == 0) return;
    ntt_list_launch(reinterpret_cast<const NttItem *>(dev + L.items), reinterpret_cast<const int *>(dev + L.p1),
                    reinterpret_cast<const int *>(dev + L.p2), L.n, L.t1, L.t2, inverse, st);
}

int launch_status()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rbk_set_error(RBK_EDEVICE, hipGetErrorString(e));
    return RBK_OK;
}

}  // namespace

extern "C" int rbk_ntt_list(rbk_ctx *c, const rbk_ntt_item *items, int n, int inverse)
{
    if (!c || n < 0 || (n > 0 && !items)) return rbk_set_error(RBK_EINVAL, "bad argument");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "list calls cannot be captured");
    if (n == 0) return RBK_OK;
    std::vector<NttItem> v((size_t)n);
    for (int i = 0; i < n; i++) {
        const rbk_ctx *ic = items[i].ctx;
        if (!ic || !items[i].d_limb) return rbk_set_error(RBK_EINVAL, "null context or limb in descriptor");
        if (ic->device != c->device) return rbk_set_error(RBK_EINVAL, "descriptor context on another device");
        if (items[i].prime < 0 || items[i].prime >= ic->nT) return rbk_set_error(RBK_EINVAL, "prime index out of range");
        if (!list_ntt_ok(ic->logN, ic->ntt_logC))
            return rbk_set_error(RBK_EUNSUPPORTED, "ring degree not supported by the list transform (N <= 2^16)");
        v[i] = NttItem{items[i].d_limb, ic->d_tabs, items[i].prime, ic->logN, ic->ntt_logC, 0};
    }
    DescBlob b;
    PackedList L = pack_list(b, v);
    int rc = RBK_OK;
    const char *dev = desc_upload(c, b, &rc);
    if (!dev) return rc;
    run_list(dev, L, inverse != 0, c->stream);
    return launch_status();
}

extern "C" int rbk_mult_relin_rescale_list(rbk_ctx *c, const uint64_t *d_a, const uint64_t *d_b, uint64_t *d_out,
                                           const int *levels, int count)
{
    if (!c || !d_a || !d_b || !d_out || !levels || count < 1) return rbk_set_error(RBK_EINVAL, "bad argument");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "list calls cannot be captured");
    if (c->nP < 1) return rbk_set_error(RBK_EUNSUPPORTED, "needs special primes (hybrid key switching)");
    if (!c->relin.data) return rbk_set_error(RBK_ENOKEY, "relinearisation key not generated");
    if (!list_ntt_ok(c->logN, c->ntt_logC))
        return rbk_set_error(RBK_EUNSUPPORTED, "ring degree not supported by the list transform (N <= 2^16)");
    int Lm = 0;
    for (int i = 0; i < count; i++) {
        if (levels[i] < 1 || levels[i] >= c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range (1..L)");
        Lm = std::max(Lm, levels[i]);
    }
    const size_t N = c->N, nP = c->nP, L1m = Lm + 1, Em = L1m + nP;
    if (ranges_overlap(d_a, (size_t)count * 2 * L1m * N, d_out, (size_t)count * 2 * Lm * N) ||
        ranges_overlap(d_b, (size_t)count * 2 * L1m * N, d_out, (size_t)count * 2 * Lm * N))
        return rbk_set_error(RBK_EINVAL, "inputs and output overlap");
    const size_t betam = (L1m + c->alpha - 1) / c->alpha;
    // ModUp tables of every level in the batch (built on first use)
    std::vector<ListCt> cts((size_t)count);
    for (int i = 0; i < count; i++) {
        const ModUpTables &T = modup_tables(c, levels[i]);
        if (!T.d_M) return rbk_set_error(RBK_ENOMEM, "ModUp tables");
        cts[i] = ListCt{levels[i], 0, T.d_A, T.d_Ash, T.d_M};
    }
    // workspace: tensor [count][3][L1m], coef [count][L1m], ext [count][betam][Em],
    // tp [count][2][nP], conv [count][2][L1m], relinearised [count][2][L1m],
    // last [count][2], lifted [count][2][Lm]  (words of N)
    const size_t cnt = count;
    const size_t w_d = cnt * 3 * L1m, w_coef = cnt * L1m, w_ext = cnt * betam * Em, w_tp = cnt * 2 * nP;
    const size_t w_conv = cnt * 2 * L1m, w_mr = cnt * 2 * L1m, w_last = cnt * 2, w_lift = cnt * 2 * Lm;
    u64 *ws = ws_reserve(c, (w_d + w_coef + w_ext + w_tp + w_conv + w_mr + w_last + w_lift) * N);
    if (!ws) return rbk_set_error(RBK_ENOMEM, "device workspace allocation failed");
    u64 *d = ws, *coef = d + w_d * N, *ext = coef + w_coef * N, *tp = ext + w_ext * N, *conv = tp + w_tp * N;
    u64 *mr = conv + w_conv * N, *last = mr + w_mr * N, *lifted = last + w_last * N;

    // descriptor lists of the five transforms with per-ciphertext shapes
    std::vector<NttItem> l_coef, l_ext, l_conv, l_last, l_lift;
    auto item = [&](u64 *p, int prime) { return NttItem{p, c->d_tabs, prime, c->logN, c->ntt_logC, 0}; };
    for (int i = 0; i < count; i++) {
        const int l = levels[i], L1 = l + 1, E = L1 + (int)nP, beta = (L1 + c->alpha - 1) / c->alpha;
        for (int limb = 0; limb < L1; limb++) l_coef.push_back(item(coef + ((size_t)i * L1m + limb) * N, limb));
        for (int j = 0; j < beta; j++) {
            const int lo = j * c->alpha, hi = std::min(L1, lo + c->alpha);
            u64 *dig = ext + ((size_t)i * betam + j) * Em * N;
            for (int pos = 0; pos < E; pos++)
                if (pos < lo || pos >= hi)
                    l_ext.push_back(item(dig + (size_t)pos * N, pos < L1 ? pos : c->nQ + pos - L1));
        }
        for (int p = 0; p < 2; p++) {
            const size_t poly = 2 * (size_t)i + p;
            for (int limb = 0; limb < L1; limb++) l_conv.push_back(item(conv + (poly * L1m + limb) * N, limb));
            l_last.push_back(item(last + poly * N, l));
            for (int limb = 0; limb < l; limb++) l_lift.push_back(item(lifted + (poly * Lm + limb) * N, limb));
        }
    }
    DescBlob b;
    const size_t o_cts = b.put(cts.data(), cts.size());
    PackedList P_coef = pack_list(b, l_coef), P_ext = pack_list(b, l_ext), P_conv = pack_list(b, l_conv);
    PackedList P_last = pack_list(b, l_last), P_lift = pack_list(b, l_lift);
    int rc = RBK_OK;
    const char *dev = desc_upload(c, b, &rc);
    if (!dev) return rc;
    const ListCt *dcts = reinterpret_cast<const ListCt *>(dev + o_cts);
    hipStream_t st = c->stream;

    // tensor product, then ModUp of d2
    tensor_list_launch(c, d_a, d_b, d, Lm, count, dcts, st);
    if (hipMemcpy2DAsync(coef, L1m * N * sizeof(u64), d + 2 * L1m * N, 3 * L1m * N * sizeof(u64), L1m * N * sizeof(u64),
                         count, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return rbk_set_error(RBK_EDEVICE, "copy failed");
    run_list(dev, P_coef, true, st);
    bconv_up_list_launch(c, coef, (long)(L1m * N), d + 2 * L1m * N, (long)(3 * L1m * N), ext, (long)(betam * Em * N),
                         (long)(Em * N), Lm, count, dcts, st);
    run_list(dev, P_ext, false, st);
    // key inner product and ModDown, plus (d0, d1)
    {
        std::vector<int> lv(count);
        for (int i = 0; i < count; i++) lv[i] = cts[i].level;
        ks_account(c, lv.data(), count, Lm);
    }
    ip_p_list_launch(c, ext, (long)(betam * Em * N), (long)(Em * N), c->relin.data, tp, Lm, count, dcts, st);
    ntt_launch(c, tp, (long)(nP * N), 2 * count, (int)nP, LimbMap{0, 0, c->nQ}, true, st);
    bconv_down_list_launch(c, tp, conv, (long)(L1m * N), Lm, count, dcts, st);
    run_list(dev, P_conv, false, st);
    moddown_ip_list_launch(c, ext, (long)(betam * Em * N), (long)(Em * N), c->relin.data, conv, (long)(2 * L1m * N),
                           (long)(L1m * N), d, (long)(3 * L1m * N), mr, (long)(2 * L1m * N), Lm, count, dcts, st);
    // rescale by each ciphertext's own last prime
    rescale_list_launch(c, 0, mr, (long)(L1m * N), last, nullptr, nullptr, 0, Lm, count, dcts, st);
    run_list(dev, P_last, true, st);
    rescale_list_launch(c, 1, nullptr, 0, last, lifted, nullptr, 0, Lm, count, dcts, st);
    run_list(dev, P_lift, false, st);
    rescale_list_launch(c, 2, mr, (long)(L1m * N), nullptr, lifted, d_out, (long)(Lm * N), Lm, count, dcts, st);
    return launch_status();
}
