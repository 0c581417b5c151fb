// Autotuner of the batched key-switching path.
//
// Three launch parameters leave every residue unchanged but move the speed:
//  * the NTT split: a limb of N = 2^logN residues is transformed as an
//    R x C matrix, C = 2^logC (column pass, then row pass); the register
//    kernels support R, C in 2^6 .. 2^8 (N = 2^13 .. 2^16); N = 2^17 takes the
//    general two-pass kernels with C = 2^8 or 2^9;
//  * the NTT chunk: how many limbs one pair of pass launches covers before
//    the next chunk starts (the intermediate of a chunk the size of the
//    memory-side cache is read back from it rather than from HBM);
//  * the ciphertexts per thread of the fused key inner products (ip_p and
//    moddown_ip): more share each key word among more ciphertexts, fewer
//    give more workgroups.
// rbk_autotune times each candidate on the shape it is asked about (level,
// batch) with HIP events on the context stream, each run starting from a
// cache overwritten by a 512 MiB scrub (as inside a pipeline), keeps the
// fastest, and
// records the choice in a text cache keyed by the GPU architecture and the
// shape, so later processes read it instead of measuring again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

namespace {

std::string tune_key(const rbk_ctx *c, int level, int count)
{
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::ostringstream os;
    os << arch << " logN=" << c->logN << " nQ=" << c->nQ << " nP=" << c->nP << " alpha=" << c->alpha
       << " level=" << level << " count=" << count;
    return os.str();
}

bool cache_lookup(const char *path, const std::string &key, int &logC, int &cpc, int &chunk)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.find(" : ");
        if (bar == std::string::npos || line.substr(0, bar) != key) continue;
        int a = 0, b = 0, k = 0;
        if (std::sscanf(line.c_str() + bar + 3, "logC=%d cpc=%d chunk=%d", &a, &b, &k) == 3) {
            logC = a;
            cpc = b;
            chunk = k;
            found = true;  // the last entry of a key wins
        }
    }
    return found;
}

// Words written before every timed run, larger than the memory-side cache:
// in a pipeline the key words and inputs of a kernel arrive from HBM, not
// from a cache a repeated run kept warm.
constexpr size_t SCRUB_WORDS = (size_t)1 << 26;  // 512 MiB

// mean ms of `reps` runs of fn after one warm-up run; each run starts after
// the scrub region has been overwritten (not timed)
template <class F>
double time_ms(rbk_ctx *c, F fn, int reps, u64 *scrub)
{
    fn();
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    const LimbMap qm{0, c->nQ, c->nQ};
    double total = 0;
    for (int i = 0; i < reps; i++) {
        ew_launch(c, EW_ZERO, scrub, nullptr, scrub, (int)(SCRUB_WORDS / c->N), 1, qm, c->stream);
        (void)hipEventRecord(e0, c->stream);
        fn();
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = -1;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < 0) {
            total = -1;
            break;
        }
        total += ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return total < 0 ? -1 : total / reps;
}

// index of the fastest candidate: every candidate is timed in each of
// `rounds` interleaved rounds (mean of `reps` runs) and keeps its best round,
// so a slow first measurement or a passing disturbance does not decide
template <class Set, class Run>
int pick_fastest(rbk_ctx *c, int n, Set set, Run run, u64 *scrub, int rounds = 3, int reps = 4)
{
    std::vector<double> best(n, 1e30);
    for (int r = 0; r < rounds; r++)
        for (int i = 0; i < n; i++) {
            set(i);
            const double ms = time_ms(c, run, reps, scrub);
            if (ms >= 0 && ms < best[i]) best[i] = ms;
        }
    int k = 0;
    for (int i = 1; i < n; i++)
        if (best[i] < best[k]) k = i;
    return k;
}

bool split_ok(int logN, int logC)
{
    const int r = logN - logC;
    if (logN == 17) return logC == 8 || logC == 9;  // general two-pass kernels (tiles of 4096 words)
    return logN >= 13 && logN <= 16 && r >= 6 && r <= 8 && logC >= 6 && logC <= 8;
}

}  // namespace

extern "C" int rbk_tune_get(const rbk_ctx *c, int *cfg)
{
    if (!c || !cfg) return rbk_set_error(RBK_EINVAL, "null argument");
    cfg[0] = c->ntt_logC;
    cfg[1] = c->ip_cpc;
    cfg[2] = c->ntt_chunk;
    return RBK_OK;
}

extern "C" int rbk_tune_set(rbk_ctx *c, const int *cfg)
{
    if (!c || !cfg) return rbk_set_error(RBK_EINVAL, "null argument");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "not allowed during graph capture");
    if (cfg[0] != c->ntt_logC && !split_ok(c->logN, cfg[0]))
        return rbk_set_error(RBK_EINVAL, "NTT split not supported for this ring degree");
    if (cfg[1] < 1 || cfg[1] > 64) return rbk_set_error(RBK_EINVAL, "ciphertexts per thread out of 1..64");
    if (cfg[2] < 0) return rbk_set_error(RBK_EINVAL, "negative NTT chunk");
    c->ntt_logC = cfg[0];
    c->ip_cpc = cfg[1];
    c->ntt_chunk = cfg[2];
    return RBK_OK;
}

extern "C" int rbk_autotune(rbk_ctx *c, int level, int count, const char *cache_path, int *cfg)
{
    if (!c || count < 1) return rbk_set_error(RBK_EINVAL, "bad argument");
    if (c->capturing) return rbk_set_error(RBK_ESTATE, "not allowed during graph capture");
    if (level < 0 || level >= c->nQ) return rbk_set_error(RBK_ELEVEL, "level out of range");
    const std::string key = tune_key(c, level, count);
    int logC = c->ntt_logC, cpc = c->ip_cpc, chunk = c->ntt_chunk;
    if (!cache_lookup(cache_path, key, logC, cpc, chunk)) {
        const size_t N = c->N, L1 = level + 1, E = L1 + c->nP, beta = (L1 + c->alpha - 1) / c->alpha;
        // scratch: the NTT batch (count x 2 polynomials) or the key-switch buffers
        const size_t ntt_words = (size_t)count * 2 * L1 * N;
        const size_t ext_words = (size_t)count * beta * E * N, conv_words = (size_t)count * 2 * L1 * N;
        const size_t tp_words = (size_t)count * 2 * c->nP * N, out_words = (size_t)count * 2 * L1 * N;
        const size_t work = std::max(ntt_words, ext_words + conv_words + tp_words + 2 * out_words);
        u64 *ws = ws_reserve(c, work + SCRUB_WORDS);
        if (!ws) return RBK_ENOMEM;
        u64 *scrub = ws + work;
        const LimbMap qm{0, c->nQ, c->nQ};
        ew_launch(c, EW_ZERO, ws, nullptr, ws, (int)(ntt_words / N), 1, qm, c->stream);
        auto ntt_pair = [&] {
            ntt_launch(c, ws, (long)(L1 * N), 2 * count, (int)L1, qm, false, c->stream);
            ntt_launch(c, ws, (long)(L1 * N), 2 * count, (int)L1, qm, true, c->stream);
        };
        // NTT split
        std::vector<int> splits;
        for (int cand = 6; cand <= 9; cand++)
            if (split_ok(c->logN, cand)) splits.push_back(cand);
        if (!splits.empty()) {
            const int k = pick_fastest(c, (int)splits.size(), [&](int i) { c->ntt_logC = splits[i]; }, ntt_pair, scrub);
            c->ntt_logC = logC = splits[k];
        }
        // NTT chunk (whole batch, or chunks around the memory-side cache size)
        const int chunks[4] = {0, 256, 512, 1024};
        const int kc = pick_fastest(c, 4, [&](int i) { c->ntt_chunk = chunks[i]; }, ntt_pair, scrub);
        c->ntt_chunk = chunk = chunks[kc];
        // ciphertexts per thread of the fused inner products (needs a key)
        // a Galois key when there is one (rotations read the digits through the automorphism)
        const DevKey *key_d = nullptr;
        for (auto &kv : c->gal)
            if (kv.second.data) {
                key_d = &kv.second;
                break;
            }
        if (!key_d && c->relin.data) key_d = &c->relin;
        if (key_d && c->nP > 0) {
            u64 *ext = ws, *conv = ext + ext_words, *tp = conv + conv_words, *out = tp + tp_words;
            u64 *c0 = out + out_words;  // the rotated input's c0, added in the epilogue
            ew_launch(c, EW_ZERO, ws, nullptr, ws, (int)((ext_words + conv_words + tp_words + 2 * out_words) / N), 1, qm,
                      c->stream);
            const u64 g = key_d->g ? key_d->g : 0;
            const int cpcs[3] = {4, 8, 16};
            // the whole ModDown of a hoisted rotation, with c0 (through the
            // automorphism) added in the epilogue: the other kernels between the
            // two inner products decide what is still cached when they run
            const int k = pick_fastest(c, 3, [&](int i) { c->ip_cpc = cpcs[i]; }, [&] {
                moddown_head_launch(c, ext, (long)(beta * E * N), key_d->data, tp, level, count, g, c->stream);
                bconv_moddown_launch(c, tp, (long)(c->nP * N), conv, (long)(L1 * N), level, 2 * count, c->stream);
                moddown_tail_launch(c, ext, (long)(beta * E * N), key_d->data, conv, c0, (long)(2 * L1 * N), g, 0, out,
                                    (long)(2 * L1 * N), level, count, g, c->stream);
            }, scrub);
            c->ip_cpc = cpc = cpcs[k];
        }
        if (hipGetLastError() != hipSuccess) return rbk_set_error(RBK_EDEVICE, "autotune launch failed");
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            if (f) f << key << " : logC=" << logC << " cpc=" << cpc << " chunk=" << chunk << "\n";
        }
    } else {
        int cfgv[3] = {logC, cpc, chunk};
        int rc = rbk_tune_set(c, cfgv);
        if (rc) return rc;
    }
    if (cfg) {
        cfg[0] = c->ntt_logC;
        cfg[1] = c->ip_cpc;
        cfg[2] = c->ntt_chunk;
    }
    return RBK_OK;
}
