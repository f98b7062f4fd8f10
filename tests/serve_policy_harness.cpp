// Host test of the request server's admission policy (serve_policy.h) against a mock
// executor: unit cases of the policy, then an event-driven simulation of a request
// stream over more systems than slots, checking after every event that the ledger
// stays within the budget and equals what the mock slots and systems actually hold,
// that requests of one system run one at a time in submission order, and that the
// queue drains.  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <vector>

#include "serve_policy.h"

using namespace labpsd;

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

static AdmitItem item(const void* sys, size_t ws64, size_t red, size_t block) {
    AdmitItem it;
    it.sys = sys;
    it.need.ws64 = ws64;
    it.need.red = red;
    it.block_bytes = block;
    return it;
}

static void unit_cases() {
    int A, B, C, D;   // system identities
    // per-system order and busy systems
    {
        Admission adm(1 << 30, 2);
        std::vector<AdmitItem> q = {item(&A, 10, 0, 8), item(&A, 10, 0, 8), item(&B, 10, 0, 8)};
        Pick p = adm.pick(q, 0);
        CHECK(p.index == 0 && !p.trim && !p.reject && p.cost == 8 * 10 + 8);
        adm.start(q[0], p, 0);
        std::vector<AdmitItem> q2 = {q[1], q[2]};
        Pick p2 = adm.pick(q2, 1);
        CHECK(p2.index == 1);   // A is busy: its second request waits, B goes first
        adm.start(q2[1], p2, 1);
        CHECK(adm.held() == 2 * (80 + 8));
        ArenaElems h;
        h.ws64 = 10;
        adm.settle(q[0], 0, h, 8);
        adm.settle(q2[1], 1, h, 8);
        CHECK(adm.held() == 2 * (80 + 8));
        // A again on slot 0: its arena and resident block are there, nothing to add
        std::vector<AdmitItem> q3 = {q[1]};
        Pick p3 = adm.pick(q3, 0);
        CHECK(p3.index == 0 && p3.cost == 0);
    }
    // a request that fits only after the idle slots give their arenas back
    {
        Admission adm(100, 2);
        AdmitItem big = item(&A, 7, 0, 4);   // 56 arena + 4 resident
        Pick p = adm.pick(std::vector<AdmitItem>{big}, 1);
        adm.start(big, p, 1);
        ArenaElems h;
        h.ws64 = 7;
        adm.settle(big, 1, h, 4);
        CHECK(adm.held() == 60);
        AdmitItem other = item(&B, 0, 5, 0);   // needs 40 of FP64 preconditioner arena on slot 0
        Pick q = adm.pick(std::vector<AdmitItem>{other}, 0);
        CHECK(q.index == 0 && !q.trim && q.cost == 40);   // 60 + 40 <= 100
        AdmitItem huge = item(&C, 10, 0, 0);               // 80 on slot 0: 140 > 100
        Pick r = adm.pick(std::vector<AdmitItem>{huge}, 0);
        CHECK(r.index == 0 && r.trim && !r.reject && r.cost == 80);   // 60 - 56 + 80 <= 100
        adm.trim_idle();
        CHECK(adm.held() == 4 && adm.have(1).bytes() == 0);
        adm.start(huge, r, 0);
        CHECK(adm.held() == 84);
    }
    // resident blocks of served systems leave too little room: reject only when every
    // slot is idle, otherwise wait
    {
        Admission adm(100, 2);
        AdmitItem a = item(&A, 0, 0, 40), b = item(&B, 0, 0, 40);
        for (const AdmitItem* it : {&a, &b}) {
            Pick p = adm.pick(std::vector<AdmitItem>{*it}, 0);
            adm.start(*it, p, 0);
            adm.settle(*it, 0, ArenaElems{}, 40);
        }
        CHECK(adm.held() == 80);
        AdmitItem c = item(&C, 3, 0, 8);   // 24 + 8 = 32: 112 > 100
        Pick p = adm.pick(std::vector<AdmitItem>{c}, 0);
        CHECK(p.index == 0 && p.reject);
        AdmitItem d = item(&D, 1, 0, 2);   // 10 fits
        Pick pd = adm.pick(std::vector<AdmitItem>{d}, 1);
        adm.start(d, pd, 1);
        Pick p2 = adm.pick(std::vector<AdmitItem>{c}, 0);
        CHECK(p2.index < 0);   // a slot runs: wait rather than reject
        // A's next request fits: its resident block is charged already
        AdmitItem a2 = item(&A, 1, 0, 40);
        Pick pa = adm.pick(std::vector<AdmitItem>{c, a2}, 0);
        CHECK(pa.index == 1 && pa.cost == 8);
    }
}

// ------------------------------------------------------------------ mock executor

struct MockReq {
    int id;
    int sys;
    AdmitItem it;
    double arrive, dur;
    double start = -1, end = -1;
    bool rejected = false;
};

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand() {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void simulation(int slots, size_t budget, int nsys, int nreq) {
    std::vector<int> sys_id(nsys);
    std::vector<size_t> sys_block(nsys), sys_ws(nsys);
    for (int s = 0; s < nsys; ++s) {
        sys_block[s] = 1 + (size_t)(urand() * 30);   // resident blocks of 1-30 units
        sys_ws[s] = 2 + (size_t)(urand() * 20);      // FP64 arena of 2-21 doubles
    }
    std::vector<MockReq> reqs(nreq);
    double t = 0;
    for (int i = 0; i < nreq; ++i) {
        t += urand() * 0.5;
        MockReq& r = reqs[i];
        r.id = i;
        r.sys = (int)(urand() * nsys);
        const bool mixed = urand() < 0.5;
        r.it.sys = &sys_id[r.sys];
        r.it.need.ws64 = sys_ws[r.sys];
        if (mixed) r.it.need.ws32 = 3 * sys_ws[r.sys];
        else r.it.need.red = sys_ws[r.sys] + 1;
        r.it.block_bytes = sys_block[r.sys];
        r.arrive = t;
        r.dur = 0.2 + urand();
    }
    Admission adm(budget, slots);
    // what the mock slots and systems really hold
    std::vector<ArenaElems> slot_mem(slots);
    std::vector<size_t> resident(nsys, 0);
    std::vector<int> slot_req(slots, -1);
    std::deque<int> queue;
    int next = 0, finished = 0, rejected = 0;
    double now = 0;
    std::map<int, int> last_started;   // per system: the last request id that started
    auto check_ledger = [&]() {
        size_t real = 0;
        for (auto& m : slot_mem) real += m.bytes();
        for (size_t v : resident) real += v;
        size_t reserved_growth = 0;   // running requests' reservations not yet settled
        for (int k = 0; k < slots; ++k)
            if (slot_req[k] >= 0) {
                const MockReq& r = reqs[slot_req[k]];
                reserved_growth += arena_growth(r.it.need, slot_mem[k]);
                const size_t res = resident[r.sys];
                reserved_growth += r.it.block_bytes > res ? r.it.block_bytes - res : 0;
            }
        CHECK(adm.held() <= budget);
        CHECK(adm.held() == real + reserved_growth);
    };
    while (finished + rejected < nreq) {
        // admit what can start now, slot by slot
        bool progress = true;
        while (progress) {
            progress = false;
            for (int k = 0; k < slots; ++k) {
                if (slot_req[k] >= 0 || queue.empty()) continue;
                std::vector<AdmitItem> items;
                for (int id : queue) items.push_back(reqs[id].it);
                const Pick p = adm.pick(items, k);
                if (p.index < 0) continue;
                const int id = queue[p.index];
                queue.erase(queue.begin() + p.index);
                MockReq& r = reqs[id];
                // its system's earlier requests have all started (submission order)
                CHECK(last_started.count(r.sys) == 0 || last_started[r.sys] < id);
                last_started[r.sys] = id;
                if (p.reject) {
                    for (int j = 0; j < slots; ++j) CHECK(slot_req[j] < 0);
                    r.rejected = true;
                    ++rejected;
                    progress = true;
                    continue;
                }
                if (p.trim) {
                    adm.trim_idle();
                    for (int j = 0; j < slots; ++j)
                        if (slot_req[j] < 0) slot_mem[j] = ArenaElems{};
                }
                for (int j = 0; j < slots; ++j)   // one request per system at a time
                    if (slot_req[j] >= 0) CHECK(reqs[slot_req[j]].sys != r.sys);
                adm.start(r.it, p, k);
                r.start = now;
                slot_req[k] = id;
                progress = true;
                check_ledger();
            }
        }
        // next event: an arrival or the earliest completion
        double t_done = 1e300;
        int k_done = -1;
        for (int k = 0; k < slots; ++k)
            if (slot_req[k] >= 0 && reqs[slot_req[k]].start + reqs[slot_req[k]].dur < t_done) {
                t_done = reqs[slot_req[k]].start + reqs[slot_req[k]].dur;
                k_done = k;
            }
        const double t_arr = next < nreq ? reqs[next].arrive : 1e300;
        if (k_done < 0 && next >= nreq) {
            CHECK(queue.empty());   // nothing runs, nothing arrives: the queue must be empty
            if (!queue.empty()) break;
        }
        if (t_arr <= t_done) {
            now = t_arr;
            queue.push_back(next++);
        } else {
            now = t_done;
            MockReq& r = reqs[slot_req[k_done]];
            // the mock solve grows the slot's arenas to the request's need and leaves a
            // resident block of the request's width
            ArenaElems& m = slot_mem[k_done];
            m.ws64 = std::max(m.ws64, r.it.need.ws64);
            m.red = std::max(m.red, r.it.need.red);
            m.ws32 = std::max(m.ws32, r.it.need.ws32);
            resident[r.sys] = std::max(resident[r.sys], r.it.block_bytes);
            adm.settle(r.it, k_done, m, resident[r.sys]);
            r.end = now;
            slot_req[k_done] = -1;
            ++finished;
            check_ledger();
        }
    }
    CHECK(finished + rejected == nreq);
    CHECK(adm.peak() <= budget);
    std::printf("simulation slots=%d budget=%zu systems=%d: %d finished, %d rejected, peak %zu\n", slots, budget,
                nsys, finished, rejected, adm.peak());
}

int main() {
    unit_cases();
    simulation(3, 4000, 12, 400);   // roomy: nothing rejected
    simulation(4, 900, 30, 600);    // tight: trimming and waiting
    simulation(4, 420, 30, 600);    // resident blocks outgrow the budget: rejections
    simulation(1, 600, 8, 200);     // one slot
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
