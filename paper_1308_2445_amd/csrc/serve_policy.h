// Admission policy of the request server (plain C++, no HIP: the host tests compile it
// with g++ against a mock executor).
//
// The server's device memory beyond the problems' own storage (H, S, the sliced-ELL
// layout, the factor) is a ledger of two kinds of bytes, both charged against the
// budget:
//   - slot arenas: every slot keeps its solve workspace between requests (the FP64 block
//     arena, the FP64 preconditioner arena, the FP32 arena) and grows it to the largest
//     request it ran; idle slots give theirs back when a queued request could not fit
//     otherwise;
//   - resident blocks: the last block of every system the server has solved (kept for the
//     next warm start), charged from its first request until the server goes away.  A
//     warm start reads the resident block in place: the solve copies its start block
//     into its own arena first and rewrites the resident block last, in stream order.
// A request is admitted on a free slot when its system is idle, it is the oldest queued
// request of that system, and the ledger plus the request's cost stays within the budget.
#pragma once

#include <cstddef>
#include <cstdint>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace labpsd {

// Elements of the three solve arenas (the layout carve() cuts them into)
struct ArenaElems {
    size_t ws64 = 0;   // doubles: the search-space blocks, Gram and Rayleigh-Ritz work
    size_t red = 0;    // doubles: FP64 preconditioner and MINRES blocks (FP64 solves)
    size_t ws32 = 0;   // floats: the same blocks in a mixed-precision solve
    size_t bytes() const { return 8 * ws64 + 8 * red + 4 * ws32; }
};

// Bytes a slot must add to hold `need` in arenas currently holding `have`.
inline size_t arena_growth(const ArenaElems& need, const ArenaElems& have) {
    auto up = [](size_t a, size_t b) { return a > b ? a - b : (size_t)0; };
    return 8 * up(need.ws64, have.ws64) + 8 * up(need.red, have.red) + 4 * up(need.ws32, have.ws32);
}

// A queued request as the policy sees it.
struct AdmitItem {
    const void* sys = nullptr;   // its system (requests of one system run in order, one at a time)
    ArenaElems need;             // its solve arenas
    size_t block_bytes = 0;      // n (nev + m0) doubles: the resident block it leaves
};

struct Ledger {
    size_t budget = 0;
    size_t held = 0;                                  // slot arenas + resident blocks
    std::unordered_map<const void*, size_t> resident;  // bytes charged per system
    size_t resident_of(const void* s) const {
        auto it = resident.find(s);
        return it == resident.end() ? 0 : it->second;
    }
};

// Bytes admitting `it` on a slot whose arenas hold `have` adds to the ledger: the arena
// growth and the growth of the system's resident block.
inline size_t admit_cost(const AdmitItem& it, const ArenaElems& have, const Ledger& L) {
    const size_t res = L.resident_of(it.sys);
    return arena_growth(it.need, have) + (it.block_bytes > res ? it.block_bytes - res : 0);
}

// Bytes a request costs on an empty slot for a system the server has not charged yet:
// larger than the budget means it can never run (ENOMEM at submission).
inline size_t standalone_cost(const AdmitItem& it) { return it.need.bytes() + it.block_bytes; }

struct Pick {
    int index = -1;       // position in the queue, -1: nothing admissible now
    bool trim = false;    // idle slots (this one included) must release their arenas first
    bool reject = false;  // the request at index can never fit: fail it (ENOMEM)
    size_t cost = 0;      // ledger bytes reserved at admission (after trimming, if any)
};

// The bookkeeping of one server: the ledger, each slot's arenas and state, the busy
// systems.  The server calls pick() and then start() or reject under its lock, releases
// the idle slots' arenas when told to trim (trim_idle() books it), and settle() with
// what the slot and the system hold after the request.
class Admission {
public:
    Admission(size_t budget, int slots) : have_(slots), running_(slots, false), res_(slots, 0), bef_(slots, 0) {
        L_.budget = budget;
    }

    // The first admissible queued request for slot k: its system idle, the oldest queued
    // request of that system, its cost within the budget (after the idle slots give back
    // their arenas if that is what it takes).  With every slot idle, a request that still
    // does not fit is rejected: only other systems' resident blocks stand in its way, and
    // they stay.
    template <class Queue>
    Pick pick(const Queue& pending, int k) const {
        size_t idle_bytes = 0;   // what trimming would give back (slot k included)
        bool all_idle = true;
        for (size_t i = 0; i < have_.size(); ++i) {
            if (!running_[i]) idle_bytes += have_[i].bytes();
            all_idle = all_idle && !running_[i];
        }
        std::unordered_set<const void*> seen;
        int idx = 0;
        for (const AdmitItem& it : pending) {
            const int here = idx++;
            if (seen.count(it.sys)) continue;   // keep each system's order
            seen.insert(it.sys);
            if (busy_.count(it.sys)) continue;
            const size_t c = admit_cost(it, have_[k], L_);
            if (L_.held + c <= L_.budget) return Pick{here, false, false, c};
            const size_t c0 = admit_cost(it, ArenaElems{}, L_);
            if (L_.held - idle_bytes + c0 <= L_.budget) return Pick{here, true, false, c0};
            if (all_idle) return Pick{here, false, true, 0};
        }
        return Pick{};
    }
    // the idle slots' arenas are given back
    void trim_idle() {
        for (size_t i = 0; i < have_.size(); ++i)
            if (!running_[i]) {
                L_.held -= have_[i].bytes();
                have_[i] = ArenaElems{};
            }
    }
    // slot k starts `it` (after pick, and trim_idle when the pick said so)
    void start(const AdmitItem& it, const Pick& pk, int k) {
        busy_.insert(it.sys);
        running_[k] = true;
        L_.held += pk.cost;
        res_[k] = pk.cost;
        bef_[k] = have_[k].bytes();
        peak_ = L_.held > peak_ ? L_.held : peak_;
    }
    // slot k finished `it`; its arenas now hold `have_after`, the system's resident block
    // is resident_after bytes
    void settle(const AdmitItem& it, int k, const ArenaElems& have_after, size_t resident_after) {
        busy_.erase(it.sys);
        running_[k] = false;
        L_.held -= res_[k];
        have_[k] = have_after;
        L_.held += have_after.bytes() - bef_[k];
        L_.held += resident_after - L_.resident_of(it.sys);
        L_.resident[it.sys] = resident_after;
        peak_ = L_.held > peak_ ? L_.held : peak_;
    }

    size_t held() const { return L_.held; }
    size_t peak() const { return peak_; }
    size_t budget() const { return L_.budget; }
    size_t resident_of(const void* sys) const { return L_.resident_of(sys); }
    const ArenaElems& have(int k) const { return have_[k]; }
    bool running(int k) const { return running_[k]; }

private:
    Ledger L_;
    std::vector<ArenaElems> have_;
    std::vector<bool> running_;
    std::vector<size_t> res_, bef_;   // per slot: bytes reserved at start, arena bytes at start
    std::unordered_set<const void*> busy_;
    size_t peak_ = 0;
};

}  // namespace labpsd
