// Admission and batching policy of the serving loop.  Plain C++17, no device
// code: the server (serve.hip) calls it under its own lock, and a CPU test
// drives it directly.
//
// * Tenants are registered with the bytes they keep resident (evaluation keys,
//   bootstrap constants); the ledger starts with them.
// * A job declares its working-set footprint.  Jobs wait in arrival order and
//   are admitted while ledger + footprint <= budget; a later job may pass a
//   head that does not fit (backfill), but only until the head has been passed
//   `max_skips` times, after which admission waits for it.
// * A tenant's next batch is its oldest admitted job plus every later admitted
//   job of the same kind and level, while the ciphertext total stays within
//   the kind's cap (max_boot_batch for bootstraps, max_batch otherwise; a first
//   job above the cap runs alone).  For a tenant registered with mixed_levels,
//   KIND_MULT jobs merge whatever their level (the server runs such batches
//   through the uneven-level list path).  Jobs of kind KIND_SOLO (a training
//   step) are never merged.
// * With cross-tenant batching on, a KIND_MULT batch of a tenant registered
//   as cross-capable also takes admitted KIND_MULT jobs of the other
//   cross-capable tenants, oldest first, within the same cap (the server runs
//   such batches through the multi-context path: every ciphertext with its
//   own tenant's keys and tables).
// * Completing a batch releases its footprints.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace rbk_sched {

enum { KIND_MULT = 1, KIND_BOOT = 2, KIND_SOLO = 3 };

struct Job {
    uint64_t id = 0;
    int tenant = 0;
    int kind = 0;
    int level = 0;
    int count = 0;
    uint64_t footprint = 0;
};

class Scheduler {
public:
    Scheduler(uint64_t budget, int max_batch, int max_boot_batch, int max_skips = 8)
        : budget_(budget),
          max_batch_(max_batch < 1 ? 1 : max_batch),
          max_boot_(max_boot_batch < 1 ? 1 : max_boot_batch),
          max_skips_(max_skips)
    {
    }

    void set_cross_tenant(bool on) { cross_ = on; }

    // false if the resident bytes do not fit next to what is already resident
    bool add_tenant(int tenant, uint64_t resident, bool mixed_levels = false, bool cross_capable = false)
    {
        if (ready_.count(tenant)) return false;
        if (resident_ + resident > budget_) return false;
        resident_ += resident;
        ledger_ += resident;
        peak_ = ledger_ > peak_ ? ledger_ : peak_;
        ready_[tenant];
        mixed_[tenant] = mixed_levels;
        cross_ok_[tenant] = cross_capable;
        return true;
    }

    // false if the tenant is unknown or the job can never fit
    bool submit(const Job &j)
    {
        if (!ready_.count(j.tenant) || j.count < 1) return false;
        if (resident_ + j.footprint > budget_) return false;
        pending_.push_back(j);
        return true;
    }

    // admit pending jobs that fit; returns them in admission order
    std::vector<Job> admit()
    {
        std::vector<Job> out;
        size_t i = 0;
        while (i < pending_.size()) {
            const Job j = pending_[i];
            if (ledger_ + j.footprint <= budget_) {
                if (i > 0) {  // passing a head that does not fit
                    if (head_skips_ >= max_skips_) break;
                    head_skips_++;
                } else {
                    head_skips_ = 0;
                }
                ledger_ += j.footprint;
                peak_ = ledger_ > peak_ ? ledger_ : peak_;
                ready_[j.tenant].push_back(j);
                out.push_back(j);
                pending_.erase(pending_.begin() + (long)i);
                continue;
            }
            if (i == 0 && head_skips_ >= max_skips_) break;
            i++;
        }
        return out;
    }

    std::vector<Job> next_batch(int tenant)
    {
        std::vector<Job> b;
        auto it = ready_.find(tenant);
        if (it == ready_.end() || it->second.empty()) return b;
        std::deque<Job> &q = it->second;
        b.push_back(q.front());
        q.pop_front();
        if (b[0].kind == KIND_SOLO) return b;
        const int cap = b[0].kind == KIND_BOOT ? max_boot_ : max_batch_;
        const bool any_level = b[0].kind == KIND_MULT && mixed_[tenant];
        int total = b[0].count;
        for (size_t k = 0; k < q.size();) {
            const Job &x = q[k];
            if (x.kind == b[0].kind && (any_level || x.level == b[0].level) && total + x.count <= cap) {
                total += x.count;
                b.push_back(x);
                q.erase(q.begin() + (long)k);
                continue;
            }
            k++;
        }
        if (cross_ && b[0].kind == KIND_MULT && cross_ok_[tenant]) {
            // other tenants' admitted mult jobs, oldest (smallest id) first
            for (;;) {
                int best_t = -1;
                size_t best_k = 0;
                uint64_t best_id = 0;
                for (auto &kv : ready_) {
                    if (kv.first == tenant || !cross_ok_[kv.first]) continue;
                    const std::deque<Job> &o = kv.second;
                    for (size_t k = 0; k < o.size(); k++)
                        if (o[k].kind == KIND_MULT && total + o[k].count <= cap && (best_t < 0 || o[k].id < best_id)) {
                            best_t = kv.first;
                            best_k = k;
                            best_id = o[k].id;
                        }
                }
                if (best_t < 0) break;
                std::deque<Job> &o = ready_[best_t];
                total += o[best_k].count;
                b.push_back(o[best_k]);
                o.erase(o.begin() + (long)best_k);
            }
        }
        return b;
    }

    void complete(const std::vector<Job> &batch)
    {
        for (const Job &j : batch) ledger_ -= j.footprint;
    }

    uint64_t ledger() const { return ledger_; }
    uint64_t peak() const { return peak_; }
    uint64_t budget() const { return budget_; }
    size_t pending() const { return pending_.size(); }
    size_t ready(int tenant) const
    {
        auto it = ready_.find(tenant);
        return it == ready_.end() ? 0 : it->second.size();
    }

private:
    uint64_t budget_, resident_ = 0, ledger_ = 0, peak_ = 0;
    int max_batch_, max_boot_, max_skips_, head_skips_ = 0;
    std::deque<Job> pending_;
    std::map<int, std::deque<Job>> ready_;
    std::map<int, bool> mixed_, cross_ok_;
    bool cross_ = false;
};

}  // namespace rbk_sched
