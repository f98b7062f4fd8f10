// Serving: a request loop over SCF-like streams of GHEPs with continuous batching.
//
// The paper solves one GHEP per SCF step, each warm-started from the previous step's
// block (Section 2; Section 3 remark 1), with S and the global factor fixed for the
// whole SCF run (Section 4).  The server keeps every system resident (H, S, the factor
// and the last block) and runs many systems' solves at once: each of max_slots slot
// threads owns a HIP stream (default priority) and executes one request at a time,
// so the kernels of concurrent requests overlap on the device.  A request is admitted
// as soon as a slot is free and its device footprint fits under the budget next to the
// requests already in flight; requests of one system keep submission order and run one
// at a time (the next warm start needs the previous result).
// Device memory: each slot owns its solve arenas (lent to the system for the duration of
// a request), so the server's memory is bounded by the ledger of serve_policy.h: slot
// arenas and the resident blocks of the systems it served, within the budget.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "common.h"


namespace labpsd {

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    Problem* sys = nullptr;
    std::vector<double> h_val;      // empty: keep H
    std::vector<double> X0;         // empty: warm start
    labpsd_solve_params prm{};
    AdmitItem item;                 // what the admission policy charges
    double t_submit = 0, t_start = 0, t_done = 0;
    bool done = false;
    labpsd_status status = LABPSD_PENDING;
    std::string error;
    std::vector<double> lambda, X;
    labpsd_stats stats{};
};

}  // namespace

struct Server {
    labpsd_ctx* ctx = nullptr;
    size_t budget = 0;
    int slots = 0;
    double t0 = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
    std::unique_ptr<Admission> adm;   // the memory ledger and the slots' states
    bool stop = false;
    uint64_t next_id = 1;
    std::vector<std::thread> workers;
    // per slot: its solve arenas
    struct Slot {
        DBuf<double> ws64, red;
        DBuf<float> ws32;
        ArenaElems have() const {
            ArenaElems a;
            a.ws64 = ws64.n;
            a.red = red.n;
            a.ws32 = ws32.n;
            return a;
        }
    };
    std::vector<std::unique_ptr<Slot>> slot;

    // The next queued request slot k starts now (mu held), or one that can never fit
    // (*reject set; the caller fails it), or nullptr.  Books the admission.
    std::shared_ptr<Request> take_admissible(int k, bool* reject) {
        *reject = false;
        std::vector<AdmitItem> items;
        items.reserve(pending.size());
        for (auto& r : pending) {
            // a resident block left by earlier solves outside the server counts at its size
            items.push_back(r->item);
            items.back().block_bytes = std::max(items.back().block_bytes, r->sys->resident_X.n * sizeof(double));
        }
        const Pick pk = adm->pick(items, k);
        if (pk.index < 0) return nullptr;
        auto it = pending.begin() + pk.index;
        auto out = *it;
        pending.erase(it);
        if (pk.reject) {
            *reject = true;
            return out;
        }
        if (pk.trim) {
            // the idle slots' arenas are not in use (their last request finished and
            // synchronised its stream); give them back
            adm->trim_idle();
            for (int i = 0; i < (int)slot.size(); ++i)
                if (!adm->running(i)) {
                    slot[i]->ws64.release();
                    slot[i]->red.release();
                    slot[i]->ws32.release();
                }
        }
        out->item = items[pk.index];
        adm->start(out->item, pk, k);
        return out;
    }

    void run_one(Request& r, Slot& sl, hipStream_t stream) {
        Problem& P = *r.sys;
        // lend the slot's arenas to the system for this solve (its own come back after)
        struct Lend {
            Problem& P;
            Slot& sl;
            Lend(Problem& p, Slot& s) : P(p), sl(s) { swap(); }
            ~Lend() { swap(); }
            void swap() {
                P.ws64.swap(sl.ws64);
                P.red.swap(sl.red);
                P.ws32.swap(sl.ws32);
            }
        } lend(P, sl);
        const int64_t n = P.n;
        const int nev = r.prm.nev, b = r.prm.nev + r.prm.m0;
        if (!r.h_val.empty()) {
            P.h_val = r.h_val;
            refresh_sell_h(P.sell, r.h_val.data(), stream);
        }
        const double* X0 = nullptr;
        labpsd_mem where = LABPSD_MEM_HOST;
        std::vector<double> E0;
        if (!r.X0.empty()) {
            X0 = r.X0.data();
        } else {
            if (P.resident_b != b || !P.resident_X.p)
                throw Error{LABPSD_EINVAL, "warm start requested but the system has no resident block of this width"};
            X0 = P.resident_X.p;
            where = LABPSD_MEM_DEVICE;
            E0 = P.resident_E;
        }
        r.lambda.assign(nev, 0.0);
        r.X.assign((size_t)n * nev, 0.0);
        // a warm start reads the resident block in place: the solve copies it into its
        // arena first and overwrites the resident block last, both on this stream
        r.status = run_solve(P, r.prm, X0, E0.empty() ? nullptr : E0.data(), where, r.lambda.data(),
                             r.X.data(), nullptr, nullptr, nullptr, LABPSD_MEM_HOST, &r.stats, stream);
    }

    void worker(int k) {
        hipStream_t stream = nullptr;
        if (hipSetDevice(ctx->device) != hipSuccess ||
            hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
            stream = nullptr;
        for (;;) {
            std::shared_ptr<Request> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                bool reject = false;
                cv_work.wait(lk, [&] {
                    if (stop) return true;
                    r = take_admissible(k, &reject);
                    return r != nullptr;
                });
                if (!r) break;   // stopping
                if (reject) {
                    r->status = LABPSD_ENOMEM;
                    r->error = "request cannot fit in the server budget next to the resident blocks of the "
                               "systems already served";
                    r->t_start = r->t_done = now_s() - t0;
                    r->done = true;
                    lk.unlock();
                    cv_done.notify_all();
                    continue;
                }
                r->t_start = now_s() - t0;
            }
            labpsd_status st = abi_guard([&]() -> labpsd_status {
                if (!stream) throw Error{LABPSD_EHIP, "slot stream could not be created"};
                run_one(*r, *slot[k], stream);
                return r->status;
            });
            {
                std::lock_guard<std::mutex> lk(mu);
                r->status = st;
                if (st < 0) r->error = get_error();
                r->t_done = now_s() - t0;
                r->done = true;
                adm->settle(r->item, k, slot[k]->have(), r->sys->resident_X.n * sizeof(double));
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (stream) (void)hipStreamDestroy(stream);
    }
};

}  // namespace labpsd

struct labpsd_server : labpsd::Server {};

using namespace labpsd;

static labpsd_status collect(labpsd_server* s, uint64_t id, double* lambda, double* X,
                             labpsd_stats* stats, double* times, bool block) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->table.find(id);
    if (it == s->table.end()) throw Error{LABPSD_EINVAL, "unknown request id"};
    std::shared_ptr<Request> r = it->second;
    if (!r->done) {
        if (!block) return LABPSD_PENDING;
        s->cv_done.wait(lk, [&] { return r->done; });
    }
    s->table.erase(id);
    lk.unlock();
    if (r->status < 0) throw Error{r->status, r->error};
    if (lambda) std::memcpy(lambda, r->lambda.data(), r->lambda.size() * sizeof(double));
    if (X) std::memcpy(X, r->X.data(), r->X.size() * sizeof(double));
    if (stats) *stats = r->stats;
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_start;
        times[2] = r->t_done;
    }
    return r->status;
}

extern "C" {

labpsd_status labpsd_server_create(labpsd_ctx* ctx, size_t hbm_budget_bytes, int max_slots,
                                   labpsd_server** out) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && out, "NULL argument");
        LABPSD_REQUIRE(max_slots >= 1 && max_slots <= 64, "max_slots must be in 1..64");
        LABPSD_REQUIRE(hbm_budget_bytes > 0, "budget must be positive");
        auto s = std::make_unique<labpsd_server>();
        s->ctx = ctx;
        s->budget = hbm_budget_bytes;
        s->adm = std::make_unique<Admission>(hbm_budget_bytes, max_slots);
        s->slots = max_slots;
        s->t0 = now_s();
        for (int i = 0; i < max_slots; ++i) s->slot.push_back(std::make_unique<Server::Slot>());
        for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([p = s.get(), i] { p->worker(i); });
        *out = s.release();
        return LABPSD_OK;
    });
}

labpsd_status labpsd_server_submit(labpsd_server* s, labpsd_problem* system, const double* h_val,
                                   const labpsd_solve_params* prm, const double* X0,
                                   uint64_t* req_id) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(s && system && prm && req_id, "NULL argument");
        if (!system->factor) throw Error{LABPSD_ESTATE, "system has no global preconditioner"};
        LABPSD_REQUIRE(prm->nev >= 1 && prm->m0 >= 0 && (int64_t)(2 * prm->nev + prm->m0) <= system->n,
                       "invalid nev / m0 for this system");
        LABPSD_REQUIRE(prm->tol > 0 && prm->max_outer >= 1 && prm->refresh_every >= 1,
                       "tol, max_outer and refresh_every must be positive");
        LABPSD_REQUIRE(prm->precision == LABPSD_FP64 || prm->precision == LABPSD_MIXED,
                       "invalid precision");
        auto r = std::make_shared<Request>();
        r->sys = system;
        r->prm = *prm;
        r->item.sys = system;
        r->item.need = solve_arena_elems(system->n, prm->nev, prm->m0, prm->precision, s->ctx->cu_count);
        r->item.block_bytes = (size_t)system->n * (prm->nev + prm->m0) * sizeof(double);
        if (standalone_cost(r->item) > s->budget)
            throw Error{LABPSD_ENOMEM, "request footprint exceeds the server budget"};
        if (h_val) r->h_val.assign(h_val, h_val + system->nnz);
        if (X0) r->X0.assign(X0, X0 + (size_t)system->n * (prm->nev + prm->m0));
        {
            std::lock_guard<std::mutex> lk(s->mu);
            LABPSD_REQUIRE(!s->stop, "server is shutting down");
            r->id = s->next_id++;
            r->t_submit = now_s() - s->t0;
            s->pending.push_back(r);
            s->table[r->id] = r;
            *req_id = r->id;
        }
        s->cv_work.notify_all();
        return LABPSD_OK;
    });
}

labpsd_status labpsd_server_poll(labpsd_server* s, uint64_t req_id, double* lambda, double* X,
                                 labpsd_stats* stats, double* times) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(s != nullptr, "NULL server");
        return collect(s, req_id, lambda, X, stats, times, false);
    });
}

labpsd_status labpsd_server_wait(labpsd_server* s, uint64_t req_id, double* lambda, double* X,
                                 labpsd_stats* stats, double* times) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(s != nullptr, "NULL server");
        return collect(s, req_id, lambda, X, stats, times, true);
    });
}

size_t labpsd_solve_footprint(int64_t n, int nev, int m0, int precision) {
    return solve_footprint_bytes(n, nev, m0, precision, 256);
}

labpsd_status labpsd_server_memory(labpsd_server* s, size_t* held, size_t* peak) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(s != nullptr, "NULL server");
        std::lock_guard<std::mutex> lk(s->mu);
        if (held) *held = s->adm->held();
        if (peak) *peak = s->adm->peak();
        return LABPSD_OK;
    });
}

void labpsd_server_destroy(labpsd_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests that never started finish as canceled
        for (auto& r : s->pending) {
            r->done = true;
            r->status = LABPSD_ESTATE;
            r->error = "server destroyed before the request started";
        }
        s->pending.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
}

}  // extern "C"
