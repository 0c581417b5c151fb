// CPU checks of the serving loop's admission and batching policy
// (paper_2506_19693_amd/csrc/serve_sched.hpp).  Prints "ok" and exits 0, or
// names the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "serve_sched.hpp"

using namespace rbk_sched;

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::printf("FAILED line %d: %s\n", __LINE__, #cond);        \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

static Job job(uint64_t id, int tenant, int kind, int level, int count, uint64_t fp)
{
    Job j;
    j.id = id;
    j.tenant = tenant;
    j.kind = kind;
    j.level = level;
    j.count = count;
    j.footprint = fp;
    return j;
}

static std::vector<uint64_t> ids(const std::vector<Job> &v)
{
    std::vector<uint64_t> r;
    for (auto &j : v) r.push_back(j.id);
    return r;
}

int main()
{
    // resident bytes count against the budget; a tenant that does not fit is refused
    {
        Scheduler s(1000, 64, 16);
        CHECK(s.add_tenant(0, 300));
        CHECK(!s.add_tenant(0, 10));  // twice
        CHECK(!s.add_tenant(1, 800));
        CHECK(s.add_tenant(1, 700));
        CHECK(s.ledger() == 1000 && s.peak() == 1000);
        CHECK(!s.submit(job(1, 0, KIND_MULT, 3, 1, 1)));  // can never fit
        CHECK(!s.submit(job(2, 7, KIND_MULT, 3, 1, 0)));  // unknown tenant
    }
    // admission in arrival order within the budget
    {
        Scheduler s(100, 64, 16);
        CHECK(s.add_tenant(0, 10));
        for (uint64_t i = 1; i <= 4; i++) CHECK(s.submit(job(i, 0, KIND_MULT, 5, 8, 30)));
        auto a = s.admit();
        CHECK((ids(a) == std::vector<uint64_t>{1, 2, 3}));
        CHECK(s.ledger() == 100 && s.pending() == 1);
        auto b = s.next_batch(0);
        CHECK((ids(b) == std::vector<uint64_t>{1, 2, 3}));  // same kind and level: one batch
        s.complete(b);
        CHECK(s.ledger() == 10);
        CHECK((ids(s.admit()) == std::vector<uint64_t>{4}));
        CHECK(s.peak() == 100);
    }
    // batches: same kind and level only, at most max_batch ciphertexts, solo jobs alone,
    // a first job above max_batch alone
    {
        Scheduler s(1 << 30, 16, 8);
        CHECK(s.add_tenant(0, 0));
        CHECK(s.add_tenant(1, 0));
        CHECK(s.submit(job(1, 0, KIND_MULT, 5, 8, 1)));
        CHECK(s.submit(job(2, 0, KIND_MULT, 6, 4, 1)));
        CHECK(s.submit(job(3, 0, KIND_BOOT, 0, 4, 1)));
        CHECK(s.submit(job(4, 0, KIND_MULT, 5, 8, 1)));
        CHECK(s.submit(job(5, 0, KIND_MULT, 5, 4, 1)));
        CHECK(s.submit(job(6, 1, KIND_MULT, 5, 4, 1)));
        CHECK(s.submit(job(7, 0, KIND_SOLO, 5, 1, 1)));
        CHECK(s.submit(job(8, 0, KIND_SOLO, 5, 1, 1)));
        CHECK(s.submit(job(9, 0, KIND_BOOT, 0, 20, 1)));
        CHECK(s.submit(job(10, 0, KIND_BOOT, 0, 2, 1)));
        CHECK(s.admit().size() == 10);
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{1, 4}));     // 8 + 8 = 16, job 5 no longer fits
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{2}));
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{3, 10}));    // 4 + 2 <= 8; job 9 (20) does not fit
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{5}));
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{7}));
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{8}));
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{9}));        // above max_batch: alone
        CHECK(s.next_batch(0).empty());
        CHECK((ids(s.next_batch(1)) == std::vector<uint64_t>{6}));        // other tenant, own queue
    }
    // a mixed-level tenant merges mult jobs of any level (bootstraps still by level)
    {
        Scheduler s(1 << 30, 16, 8);
        CHECK(s.add_tenant(0, 0, true));
        CHECK(s.add_tenant(1, 0, false));
        CHECK(s.submit(job(1, 0, KIND_MULT, 5, 4, 1)));
        CHECK(s.submit(job(2, 0, KIND_MULT, 9, 4, 1)));
        CHECK(s.submit(job(3, 0, KIND_BOOT, 0, 2, 1)));
        CHECK(s.submit(job(4, 0, KIND_BOOT, 1, 2, 1)));
        CHECK(s.submit(job(5, 0, KIND_MULT, 2, 10, 1)));
        CHECK(s.submit(job(6, 1, KIND_MULT, 5, 4, 1)));
        CHECK(s.submit(job(7, 1, KIND_MULT, 9, 4, 1)));
        CHECK(s.admit().size() == 7);
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{1, 2}));     // levels 5 and 9 together; 18 > 16
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{3}));        // bootstraps: same level only
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{4}));
        CHECK((ids(s.next_batch(0)) == std::vector<uint64_t>{5}));
        CHECK((ids(s.next_batch(1)) == std::vector<uint64_t>{6}));        // not mixed: by level
        CHECK((ids(s.next_batch(1)) == std::vector<uint64_t>{7}));
    }
    // backfill past a head that does not fit, bounded by max_skips
    {
        Scheduler s(100, 64, 16, 3);
        CHECK(s.add_tenant(0, 0));
        CHECK(s.submit(job(1, 0, KIND_MULT, 5, 1, 60)));
        CHECK((ids(s.admit()) == std::vector<uint64_t>{1}));
        CHECK(s.submit(job(2, 0, KIND_MULT, 5, 1, 70)));  // head, waits for job 1
        for (uint64_t i = 3; i <= 8; i++) CHECK(s.submit(job(i, 0, KIND_MULT, 5, 1, 10)));
        auto a = s.admit();
        CHECK((ids(a) == std::vector<uint64_t>{3, 4, 5}));  // three passes, then the head blocks
        CHECK(s.admit().empty());
        CHECK(s.ledger() == 90);
        auto b1 = s.next_batch(0);  // jobs 1, 3, 4, 5 run together
        CHECK(b1.size() == 4);
        s.complete(b1);
        CHECK((ids(s.admit()) == std::vector<uint64_t>{2, 6, 7, 8}));
        CHECK(s.ledger() == 100);
    }
    // random traffic: the ledger never exceeds the budget, every job is admitted
    // and completed exactly once, batches are homogeneous and bounded
    {
        std::mt19937_64 rng(7);
        const uint64_t budget = 5000;
        const int max_batch = 32, max_boot = 12;
        Scheduler s(budget, max_batch, max_boot, 4);
        const int tenants = 4;
        for (int t = 0; t < tenants; t++) CHECK(s.add_tenant(t, 200));
        std::set<uint64_t> submitted, admitted, completed;
        std::vector<std::vector<Job>> running;
        uint64_t next = 1;
        for (int round = 0; round < 4000; round++) {
            const int act = (int)(rng() % 3);
            if (act == 0 && next <= 1500) {
                int kind = 1 + (int)(rng() % 3);
                int count = kind == KIND_SOLO ? 1 : 1 + (int)(rng() % 40);
                Job j = job(next, (int)(rng() % tenants), kind, kind == KIND_BOOT ? 0 : 1 + (int)(rng() % 4), count,
                            50 + rng() % 3000);
                CHECK(s.submit(j));
                submitted.insert(next++);
            } else if (act == 1) {
                int t = (int)(rng() % tenants);
                auto b = s.next_batch(t);
                if (!b.empty()) {
                    int total = 0;
                    for (auto &x : b) {
                        CHECK(x.tenant == t && x.kind == b[0].kind && x.level == b[0].level);
                        CHECK(admitted.count(x.id));
                        total += x.count;
                    }
                    CHECK(b.size() == 1 || total <= (b[0].kind == KIND_BOOT ? max_boot : max_batch));
                    CHECK(b[0].kind != KIND_SOLO || b.size() == 1);
                    running.push_back(b);
                }
            } else if (!running.empty()) {
                size_t k = rng() % running.size();
                for (auto &x : running[k]) CHECK(completed.insert(x.id).second);
                s.complete(running[k]);
                running.erase(running.begin() + (long)k);
            }
            for (auto &x : s.admit()) CHECK(admitted.insert(x.id).second);
            CHECK(s.ledger() <= budget);
        }
        // drain
        for (int guard = 0; guard < 100000 && completed.size() < submitted.size(); guard++) {
            for (auto &b : running) {
                for (auto &x : b) CHECK(completed.insert(x.id).second);
                s.complete(b);
            }
            running.clear();
            for (auto &x : s.admit()) CHECK(admitted.insert(x.id).second);
            for (int t = 0; t < tenants; t++) {
                auto b = s.next_batch(t);
                if (!b.empty()) running.push_back(b);
            }
            CHECK(s.ledger() <= budget);
        }
        CHECK(completed == submitted && admitted == submitted);
        CHECK(s.ledger() == 200 * tenants);
        CHECK(s.peak() <= budget);
    }
    // cross-tenant batching: mult jobs of other cross-capable tenants join, oldest first, within the cap;
    // bootstraps, training steps and tenants that are not cross-capable never do
    {
        Scheduler s(1 << 20, 32, 16);
        s.set_cross_tenant(true);
        CHECK(s.add_tenant(0, 0, true, true));
        CHECK(s.add_tenant(1, 0, true, true));
        CHECK(s.add_tenant(2, 0, true, false));
        CHECK(s.submit(job(1, 0, KIND_MULT, 5, 8, 1)));
        CHECK(s.submit(job(2, 1, KIND_MULT, 9, 16, 1)));
        CHECK(s.submit(job(3, 2, KIND_MULT, 5, 4, 1)));
        CHECK(s.submit(job(4, 1, KIND_BOOT, 0, 2, 1)));
        CHECK(s.submit(job(5, 1, KIND_MULT, 7, 8, 1)));
        CHECK(s.submit(job(6, 1, KIND_MULT, 7, 4, 1)));
        CHECK(s.admit().size() == 6);
        auto b = s.next_batch(0);
        CHECK(ids(b) == (std::vector<uint64_t>{1, 2, 5}));    // 8 + 16 + 8 = 32; job 6 does not fit
        CHECK(s.ready(1) == 2 && s.ready(2) == 1);
        auto b1 = s.next_batch(1);
        CHECK(ids(b1) == (std::vector<uint64_t>{4}));          // a bootstrap head merges with nothing here
        auto b2 = s.next_batch(1);
        CHECK(ids(b2) == (std::vector<uint64_t>{6}));          // tenant 2 is not cross-capable
        CHECK(ids(s.next_batch(2)) == (std::vector<uint64_t>{3}));
    }
    // off by default
    {
        Scheduler s(1 << 20, 32, 16);
        CHECK(s.add_tenant(0, 0, true, true));
        CHECK(s.add_tenant(1, 0, true, true));
        CHECK(s.submit(job(1, 0, KIND_MULT, 5, 8, 1)));
        CHECK(s.submit(job(2, 1, KIND_MULT, 5, 8, 1)));
        CHECK(s.admit().size() == 2);
        CHECK(ids(s.next_batch(0)) == (std::vector<uint64_t>{1}));
    }
    std::printf("ok\n");
    return 0;
}
