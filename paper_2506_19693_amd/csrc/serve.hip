// Serving loop: encrypted-training jobs of several tenants on one GPU.
//
// Each tenant is a context (its parameters and evaluation keys, resident in
// HBM) that the server drives from a worker thread of its own, on a HIP
// stream of its own, so the work of different tenants overlaps on the
// device.  Jobs are admitted by memory footprint against an HBM ledger that
// starts with every tenant's resident bytes (serve_sched.hpp).  Each time a
// tenant's stream is free, its worker takes the oldest admitted job plus every
// queued job it can merge with (same kind and level, up to max_batch
// ciphertexts) and runs them as one batched launch set: inputs are gathered
// into a staging batch, the batched entry point runs once, results are
// scattered back.  The batched entry points compute exactly what the
// per-ciphertext ones do, so a job's result does not depend on what it was
// batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"
#include "serve_sched.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct SJob {
    rbk_job j{};
    std::vector<double> scales_in;
    Clock::time_point t_submit, t_admit, t_start, t_end;
    int status = 0;
    std::string msg;
    int batch_cts = 0;
    bool admitted = false, done = false;
};

struct Tenant {
    int id = 0;
    rbk_ctx *c = nullptr;
    hipStream_t st = nullptr;
    hipStream_t old_stream = nullptr;
    int old_lanes = 1;
    uint64_t resident = 0;
    std::thread th;
    u64 *stage = nullptr;
    size_t stage_words = 0;
};

size_t ct_words(const rbk_ctx *c, int level) { return (size_t)2 * (level + 1) * c->N; }

uint64_t key_bytes(const rbk_ctx *c)
{
    const uint64_t one = (uint64_t)c->beta * 2 * c->nT * c->N * sizeof(u64);
    uint64_t n = c->relin.data ? 1 : 0;
    for (auto &kv : c->gal)
        if (kv.second.data) n++;
    return n * one;
}

}  // namespace

struct rbk_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    rbk_sched::Scheduler sched;
    std::map<uint64_t, SJob> jobs;
    std::vector<Tenant *> tenants;
    uint64_t next_id = 1;
    bool running = false, stopping = false;
    uint64_t n_batches = 0, n_jobs_done = 0, n_merged = 0, n_outstanding = 0, n_cross = 0;
    int max_batch, max_boot;
    bool cross = false;

    rbk_server(uint64_t budget, int mb, int mbb) : sched(budget, mb, mbb), max_batch(mb), max_boot(mbb) {}
};

namespace {

// mult jobs of any level share batches (the uneven-level list path) when the
// context supports it: hybrid key switching and a ring degree up to 2^16
bool mixed_levels(const rbk_ctx *c)
{
    if (c->nP < 1) return false;
    if (c->logN <= 12) return true;
    const int r = c->logN - c->ntt_logC;
    return c->logN <= 16 && r >= 6 && r <= 8 && c->ntt_logC >= 6 && c->ntt_logC <= 8;
}

// working-set estimate of a job, bytes (admission only; see rbk.h).  Jobs run
// in chunks of at most max_batch (mult) / max_boot (bootstrap) ciphertexts.
// A mult job of a mixed-level tenant may share a chunk with ciphertexts of
// the top level, whose slot strides the whole chunk then uses: its working
// set is counted at the top level.
uint64_t footprint(const rbk_ctx *c, const rbk_job &j, int max_batch, int max_boot)
{
    const uint64_t w8 = sizeof(u64);
    switch (j.kind) {
    case RBK_JOB_MULT_RESCALE: {
        const int wl = mixed_levels(c) ? c->nQ - 1 : j.level;
        const uint64_t ct = ct_words(c, j.level), cw = ct_words(c, wl), n = (uint64_t)std::min(j.count, max_batch);
        return w8 * ((uint64_t)j.count * ct + n * (2 * cw + 3 * cw / 2 + cw + cw) + ks_words(c, wl, (int)n));
    }
    case RBK_JOB_BOOTSTRAP:
        return w8 * (uint64_t)std::min(j.count, max_boot) * 48 * ct_words(c, c->nQ - 1);
    case RBK_JOB_TRAIN_STEP:
        return w8 * (uint64_t)j.b * 24 * ct_words(c, j.level) + w8 * ks_words(c, j.level, j.b);
    default:
        return 0;
    }
}

u64 *stage_reserve(Tenant *t, size_t words)
{
    if (words <= t->stage_words) return t->stage;
    if (t->stage) {
        (void)hipStreamSynchronize(t->st);
        (void)hipFree(t->stage);
        t->stage = nullptr;
        t->stage_words = 0;
    }
    if (hipMalloc((void **)&t->stage, words * sizeof(u64)) != hipSuccess) return nullptr;
    t->stage_words = words;
    return t->stage;
}

// copy limbs 0..level of every polynomial of count ciphertexts laid out at
// in_level into a batch whose slots are laid out at slot_level (default: level)
int gather(Tenant *t, const uint64_t *src, int in_level, int level, int count, u64 *dst, int slot_level = -1)
{
    const rbk_ctx *c = t->c;
    if (slot_level < 0) slot_level = level;
    const size_t N = c->N, w = (size_t)(level + 1) * N, sp = (size_t)(in_level + 1) * N;
    const size_t dp = (size_t)(slot_level + 1) * N;
    if (hipMemcpy2DAsync(dst, dp * sizeof(u64), src, sp * sizeof(u64), w * sizeof(u64), (size_t)2 * count,
                         hipMemcpyDeviceToDevice, t->st) != hipSuccess)
        return rbk_set_error(RBK_EDEVICE, "gather copy failed");
    return RBK_OK;
}

// the ciphertexts of a batch, job by job, as (job, first index, count) pieces
// of chunks of at most `cap`
struct Piece {
    SJob *s;
    int first, n;
};

std::vector<std::vector<Piece>> chunks(std::vector<SJob *> &b, int cap)
{
    std::vector<std::vector<Piece>> out(1);
    int fill = 0;
    for (SJob *s : b) {
        for (int i = 0; i < s->j.count;) {
            if (fill == cap) {
                out.emplace_back();
                fill = 0;
            }
            const int n = std::min(s->j.count - i, cap - fill);
            out.back().push_back(Piece{s, i, n});
            fill += n;
            i += n;
        }
    }
    return out;
}

// a batch of mult jobs at uneven levels: slots at the chunk's largest level,
// one uneven-level list call per chunk
int run_mult_list(Tenant *t, std::vector<SJob *> &b, int cap)
{
    rbk_ctx *c = t->c;
    const size_t N = c->N;
    for (auto &ch : chunks(b, cap)) {
        int total = 0, Lm = 0, rc;
        std::vector<int> levels;
        for (auto &p : ch) {
            total += p.n;
            Lm = std::max(Lm, p.s->j.level);
            levels.insert(levels.end(), (size_t)p.n, p.s->j.level);
        }
        const size_t ct = ct_words(c, Lm), ct_out = ct_words(c, Lm - 1);
        u64 *A = stage_reserve(t, (size_t)total * (2 * ct + ct_out));
        if (!A) return rbk_set_error(RBK_ENOMEM, "staging allocation failed");
        u64 *B = A + (size_t)total * ct, *R = B + (size_t)total * ct;
        int off = 0;
        for (auto &p : ch) {
            const rbk_job &j = p.s->j;
            const size_t in_ct = ct_words(c, j.in_level);
            if ((rc = gather(t, j.d_a + p.first * in_ct, j.in_level, j.level, p.n, A + (size_t)off * ct, Lm))) return rc;
            if ((rc = gather(t, j.d_b + p.first * in_ct, j.in_level, j.level, p.n, B + (size_t)off * ct, Lm))) return rc;
            off += p.n;
        }
        if ((rc = rbk_mult_relin_rescale_list(c, A, B, R, levels.data(), total))) return rc;
        off = 0;
        for (auto &p : ch) {
            // limbs 0..l-1 of each polynomial from slots of Lm limbs
            const int l = p.s->j.level;
            const size_t w = (size_t)l * N;
            if (hipMemcpy2DAsync(p.s->j.d_out + p.first * ct_words(c, l - 1), w * sizeof(u64),
                                 R + (size_t)off * ct_out, (size_t)Lm * N * sizeof(u64), w * sizeof(u64),
                                 (size_t)2 * p.n, hipMemcpyDeviceToDevice, t->st) != hipSuccess)
                return rbk_set_error(RBK_EDEVICE, "scatter copy failed");
            off += p.n;
        }
    }
    return RBK_OK;
}

// A mult batch holding other tenants' jobs: every ciphertext runs in its own
// tenant's context (keys, tables) through one multi-context call per chunk,
// on this worker's stream and workspace; results go straight to the jobs'
// outputs.  The other contexts are only read (their ModUp tables were built
// before the workers started).
int run_mult_multi(rbk_server *S, Tenant *t, std::vector<SJob *> &b, int cap)
{
    for (auto &ch : chunks(b, cap)) {
        size_t words = 0;
        for (auto &p : ch) words += (size_t)p.n * 2 * ct_words(S->tenants[p.s->j.tenant]->c, p.s->j.level);
        u64 *A = stage_reserve(t, words);
        if (!A) return rbk_set_error(RBK_ENOMEM, "staging allocation failed");
        std::vector<rbk_mr_item> items;
        size_t off = 0;
        for (auto &p : ch) {
            const rbk_job &j = p.s->j;
            rbk_ctx *uc = S->tenants[j.tenant]->c;
            const size_t N = uc->N, ct = ct_words(uc, j.level), in_ct = ct_words(uc, j.in_level);
            const size_t out_ct = ct_words(uc, j.level - 1), w = (size_t)(j.level + 1) * N;
            u64 *Ap = A + off, *Bp = Ap + (size_t)p.n * ct;
            // limbs 0..level of every polynomial, from inputs laid out at in_level
            if (hipMemcpy2DAsync(Ap, w * sizeof(u64), j.d_a + p.first * in_ct, (size_t)(j.in_level + 1) * N * sizeof(u64),
                                 w * sizeof(u64), (size_t)2 * p.n, hipMemcpyDeviceToDevice, t->st) != hipSuccess ||
                hipMemcpy2DAsync(Bp, w * sizeof(u64), j.d_b + p.first * in_ct, (size_t)(j.in_level + 1) * N * sizeof(u64),
                                 w * sizeof(u64), (size_t)2 * p.n, hipMemcpyDeviceToDevice, t->st) != hipSuccess)
                return rbk_set_error(RBK_EDEVICE, "gather copy failed");
            for (int i = 0; i < p.n; i++)
                items.push_back(rbk_mr_item{uc, Ap + i * ct, Bp + i * ct, j.d_out + (p.first + i) * out_ct, j.level, 0});
            off += (size_t)p.n * 2 * ct;
        }
        if (int rc = rbk_mult_relin_rescale_multi(t->c, items.data(), (int)items.size())) return rc;
    }
    return RBK_OK;
}

int run_mult(Tenant *t, std::vector<SJob *> &b, int cap)
{
    rbk_ctx *c = t->c;
    for (SJob *s : b)
        if (s->j.level != b[0]->j.level) return run_mult_list(t, b, cap);
    const int lv = b[0]->j.level;
    const size_t ct = ct_words(c, lv), ct_out = ct_words(c, lv - 1);
    for (auto &ch : chunks(b, cap)) {
        int total = 0, rc;
        for (auto &p : ch) total += p.n;
        u64 *A = stage_reserve(t, (size_t)total * (3 * ct) + (size_t)total * ct_out);
        if (!A) return rbk_set_error(RBK_ENOMEM, "staging allocation failed");
        u64 *B = A + (size_t)total * ct, *M = B + (size_t)total * ct, *R = M + (size_t)total * ct;
        int off = 0;
        for (auto &p : ch) {
            const rbk_job &j = p.s->j;
            const size_t in_ct = ct_words(c, j.in_level);
            if ((rc = gather(t, j.d_a + p.first * in_ct, j.in_level, lv, p.n, A + (size_t)off * ct))) return rc;
            if ((rc = gather(t, j.d_b + p.first * in_ct, j.in_level, lv, p.n, B + (size_t)off * ct))) return rc;
            off += p.n;
        }
        if ((rc = rbk_mult_relin_batch(c, A, B, M, lv, total))) return rc;
        if ((rc = rbk_rescale_batch(c, M, R, lv, total))) return rc;
        off = 0;
        for (auto &p : ch) {
            if (hipMemcpyAsync(p.s->j.d_out + p.first * ct_out, R + (size_t)off * ct_out, (size_t)p.n * ct_out * sizeof(u64),
                               hipMemcpyDeviceToDevice, t->st) != hipSuccess)
                return rbk_set_error(RBK_EDEVICE, "scatter copy failed");
            off += p.n;
        }
    }
    return RBK_OK;
}

int run_boot(Tenant *t, std::vector<SJob *> &b, int cap)
{
    rbk_ctx *c = t->c;
    int levels[4], np = 0, ns = 0, rc;
    if ((rc = rbk_boot_info(c, levels, &np, &ns))) return rc;
    const int lo = levels[3];
    const size_t ci = ct_words(c, 0), co = ct_words(c, lo);
    for (auto &ch : chunks(b, cap)) {
        int total = 0;
        for (auto &p : ch) total += p.n;
        u64 *I = stage_reserve(t, (size_t)total * (ci + co));
        if (!I) return rbk_set_error(RBK_ENOMEM, "staging allocation failed");
        u64 *O = I + (size_t)total * ci;
        std::vector<double> sin, sout(total);
        int off = 0;
        for (auto &p : ch) {
            const rbk_job &j = p.s->j;
            const size_t in_ct = ct_words(c, j.in_level);
            if ((rc = gather(t, j.d_a + p.first * in_ct, j.in_level, 0, p.n, I + (size_t)off * ci))) return rc;
            sin.insert(sin.end(), p.s->scales_in.begin() + p.first, p.s->scales_in.begin() + p.first + p.n);
            off += p.n;
        }
        if ((rc = rbk_bootstrap_batch(c, I, sin.data(), O, sout.data(), total))) return rc;
        off = 0;
        for (auto &p : ch) {
            if (hipMemcpyAsync(p.s->j.d_out + p.first * co, O + (size_t)off * co, (size_t)p.n * co * sizeof(u64),
                               hipMemcpyDeviceToDevice, t->st) != hipSuccess)
                return rbk_set_error(RBK_EDEVICE, "scatter copy failed");
            if (p.s->j.scales_out)
                for (int i = 0; i < p.n; i++) p.s->j.scales_out[p.first + i] = sout[off + i];
            off += p.n;
        }
    }
    return RBK_OK;
}

int run_train(Tenant *, std::vector<SJob *> &b)
{
    const rbk_job &j = b[0]->j;
    for (int s = 0; s < j.count; s++) {
        // one stream, like every served call (the footprint has no side-stream workspace)
        int rc = rbk_mlp_train_step(j.mlp, j.d_x, j.d_y_exp, j.d_y_rep, j.b, j.level, j.scale, j.t0 + s,
                                    RBK_MLP_SEQUENTIAL);
        if (rc) return rc;
    }
    return RBK_OK;
}

void worker(rbk_server *S, Tenant *t)
{
    hipSetDevice(t->c->device);
    for (;;) {
        std::vector<rbk_sched::Job> batch;
        std::vector<SJob *> sj;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // a stopping server still runs every job already submitted
            S->cv_work.wait(lk, [&] {
                return S->sched.ready(t->id) > 0 || (S->stopping && S->sched.pending() == 0);
            });
            if (S->sched.ready(t->id) == 0) return;
            batch = S->sched.next_batch(t->id);
            const auto now = Clock::now();
            int cts = 0;
            for (auto &x : batch) cts += x.count;
            for (auto &x : batch) {
                SJob &s = S->jobs[x.id];
                s.t_start = now;
                s.batch_cts = cts;
                sj.push_back(&s);
            }
        }
        int rc, foreign = 0;
        for (SJob *x : sj) foreign += x->j.tenant != t->id;
        switch (sj[0]->j.kind) {
        case RBK_JOB_MULT_RESCALE:
            rc = foreign ? run_mult_multi(S, t, sj, S->max_batch) : run_mult(t, sj, S->max_batch);
            break;
        case RBK_JOB_BOOTSTRAP: rc = run_boot(t, sj, S->max_boot); break;
        default: rc = run_train(t, sj); break;
        }
        if (hipStreamSynchronize(t->st) != hipSuccess && !rc) rc = rbk_set_error(RBK_EDEVICE, "stream failed");
        const std::string msg = rc ? rbk_last_error() : "";
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const auto now = Clock::now();
            for (SJob *s : sj) {
                s->status = rc;
                s->msg = msg;
                s->t_end = now;
                s->done = true;
            }
            S->n_outstanding -= sj.size();
            S->sched.complete(batch);
            S->n_batches++;
            S->n_jobs_done += batch.size();
            if (batch.size() > 1) S->n_merged += batch.size();
            S->n_cross += foreign;
            for (auto &x : S->sched.admit()) {
                S->jobs[x.id].admitted = true;
                S->jobs[x.id].t_admit = now;
            }
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" int rbk_server_create(uint64_t hbm_budget, int max_batch, int max_boot_batch, rbk_server **out)
{
    if (!out || hbm_budget == 0 || max_batch < 1 || max_boot_batch < 1) return rbk_set_error(RBK_EINVAL, "bad argument");
    *out = new (std::nothrow) rbk_server(hbm_budget, max_batch, max_boot_batch);
    return *out ? RBK_OK : rbk_set_error(RBK_ENOMEM, "host allocation failed");
}

extern "C" int rbk_server_add_tenant(rbk_server *S, rbk_ctx *c, int *tenant)
{
    if (!S || !c || !tenant) return rbk_set_error(RBK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) return rbk_set_error(RBK_ESTATE, "tenants are added before rbk_server_start");
    for (Tenant *t : S->tenants)
        if (t->c == c) return rbk_set_error(RBK_EINVAL, "context already registered");
    Tenant *t = new Tenant;
    t->id = (int)S->tenants.size();
    t->c = c;
    t->resident = key_bytes(c) + boot_resident_bytes(c);
    if (!S->sched.add_tenant(t->id, t->resident, mixed_levels(c), mixed_levels(c))) {
        delete t;
        return rbk_set_error(RBK_ENOMEM, "the tenant's resident keys do not fit the HBM budget");
    }
    if (hipSetDevice(c->device) != hipSuccess || hipStreamCreateWithFlags(&t->st, hipStreamNonBlocking) != hipSuccess) {
        delete t;
        return rbk_set_error(RBK_EDEVICE, "stream creation failed");
    }
    t->old_stream = c->stream;
    c->stream = t->st;
    // a served context runs on one lane: the tenants' streams overlap each
    // other instead, and the footprints the ledger admits by assume no lane
    // buffers
    t->old_lanes = c->lanes;
    c->lanes = 1;
    S->tenants.push_back(t);
    *tenant = t->id;
    return RBK_OK;
}

extern "C" int rbk_server_start(rbk_server *S)
{
    if (!S) return rbk_set_error(RBK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) return RBK_OK;
    if (S->cross) {
        // other workers read these tables: build every level now, so later lookups only read
        for (Tenant *t : S->tenants) {
            if (!mixed_levels(t->c)) continue;
            if (hipSetDevice(t->c->device) != hipSuccess) return rbk_set_error(RBK_EDEVICE, "hipSetDevice failed");
            for (int l = 1; l < t->c->nQ; l++)
                if (!modup_tables(t->c, l).d_M) return rbk_set_error(RBK_ENOMEM, "ModUp tables");
        }
    }
    S->running = true;
    for (Tenant *t : S->tenants) t->th = std::thread(worker, S, t);
    return RBK_OK;
}

extern "C" int rbk_server_set_cross_tenant(rbk_server *S, int on)
{
    if (!S) return rbk_set_error(RBK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) return rbk_set_error(RBK_ESTATE, "set before rbk_server_start");
    S->cross = on != 0;
    S->sched.set_cross_tenant(S->cross);
    return RBK_OK;
}

extern "C" int rbk_server_cross_merged(rbk_server *S, uint64_t *n)
{
    if (!S || !n) return rbk_set_error(RBK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *n = S->n_cross;
    return RBK_OK;
}

extern "C" int rbk_server_submit(rbk_server *S, const rbk_job *j, uint64_t *id)
{
    if (!S || !j || !id) return rbk_set_error(RBK_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->running || S->stopping) return rbk_set_error(RBK_ESTATE, "server not running");
    if (j->tenant < 0 || j->tenant >= (int)S->tenants.size()) return rbk_set_error(RBK_EINVAL, "unknown tenant");
    const rbk_ctx *c = S->tenants[j->tenant]->c;
    int kind;
    switch (j->kind) {
    case RBK_JOB_MULT_RESCALE:
        if (j->count < 1 || !j->d_a || !j->d_b || !j->d_out) return rbk_set_error(RBK_EINVAL, "bad mult job");
        if (j->level < 1 || j->in_level < j->level || j->in_level >= c->nQ)
            return rbk_set_error(RBK_ELEVEL, "bad mult job levels");
        kind = rbk_sched::KIND_MULT;
        break;
    case RBK_JOB_BOOTSTRAP:
        if (j->count < 1 || !j->d_a || !j->d_out || !j->scales_in) return rbk_set_error(RBK_EINVAL, "bad bootstrap job");
        if (!c->boot) return rbk_set_error(RBK_ESTATE, "tenant has no bootstrap plan");
        if (j->in_level < 0 || j->in_level >= c->nQ) return rbk_set_error(RBK_ELEVEL, "bad bootstrap input level");
        kind = rbk_sched::KIND_BOOT;
        break;
    case RBK_JOB_TRAIN_STEP:
        if (j->count < 1 || !j->mlp || !j->d_x || !j->d_y_exp || !j->d_y_rep || j->b < 1 || j->t0 < 1)
            return rbk_set_error(RBK_EINVAL, "bad train job");
        if (j->level < 0 || j->level >= c->nQ) return rbk_set_error(RBK_ELEVEL, "bad train job level");
        kind = rbk_sched::KIND_SOLO;
        break;
    default:
        return rbk_set_error(RBK_EINVAL, "unknown job kind");
    }
    rbk_sched::Job sj;
    sj.id = S->next_id++;
    sj.tenant = j->tenant;
    sj.kind = kind;
    sj.level = j->kind == RBK_JOB_BOOTSTRAP ? 0 : j->level;
    sj.count = j->kind == RBK_JOB_TRAIN_STEP ? 1 : j->count;
    sj.footprint = footprint(c, *j, S->max_batch, S->max_boot);
    if (!S->sched.submit(sj)) return rbk_set_error(RBK_ENOMEM, "job footprint exceeds the HBM budget");
    SJob &s = S->jobs[sj.id];
    s.j = *j;
    if (j->kind == RBK_JOB_BOOTSTRAP) s.scales_in.assign(j->scales_in, j->scales_in + j->count);
    s.t_submit = Clock::now();
    S->n_outstanding++;
    for (auto &x : S->sched.admit()) {
        S->jobs[x.id].admitted = true;
        S->jobs[x.id].t_admit = s.t_submit;
    }
    *id = sj.id;
    lk.unlock();
    S->cv_work.notify_all();
    return RBK_OK;
}

extern "C" int rbk_server_wait(rbk_server *S, uint64_t id, rbk_job_result *res)
{
    if (!S || !res) return rbk_set_error(RBK_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return rbk_set_error(RBK_EINVAL, "unknown job id");
    S->cv_done.wait(lk, [&] { return it->second.done; });
    const SJob &s = it->second;
    res->status = s.status;
    res->latency_ms = ms_between(s.t_submit, s.t_end);
    res->queue_ms = ms_between(s.t_submit, s.t_start);
    res->run_ms = ms_between(s.t_start, s.t_end);
    res->batch_cts = s.batch_cts;
    const int st = s.status;
    const std::string msg = s.msg;
    S->jobs.erase(it);
    if (st) return rbk_set_error(st, msg.c_str());
    return RBK_OK;
}

extern "C" int rbk_server_drain(rbk_server *S)
{
    if (!S) return rbk_set_error(RBK_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->n_outstanding == 0; });
    return RBK_OK;
}

extern "C" int rbk_server_stats(rbk_server *S, uint64_t *stats)
{
    if (!S || !stats) return rbk_set_error(RBK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    stats[0] = S->n_jobs_done;
    stats[1] = S->n_batches;
    stats[2] = S->n_merged;
    stats[3] = S->sched.peak();
    stats[4] = S->sched.ledger();
    stats[5] = S->sched.budget();
    return RBK_OK;
}

extern "C" int rbk_server_destroy(rbk_server *S)
{
    if (!S) return RBK_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (Tenant *t : S->tenants) {
        if (t->th.joinable()) t->th.join();
        (void)hipStreamSynchronize(t->st);
        if (t->stage) (void)hipFree(t->stage);
        t->c->stream = t->old_stream;
        t->c->lanes = t->old_lanes;
        (void)hipStreamDestroy(t->st);
        delete t;
    }
    delete S;
    return RBK_OK;
}
