// Host check of the server's admission pass (admission.h), built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitized.py.
// Seeded random arrivals and completions of forward and inversion requests
// against a slot count per kind and a byte budget; after every pass the
// started and waiting requests are checked against the policy from outside:
//  * started requests of each kind keep arrival order, and the waiting queue
//    keeps its order;
//  * a request is passed over by a later one only if it is an inversion and
//    no inversion slot is free (forward requests passing such inversions);
//  * the pass ends only where the policy says it must: walking the waiting
//    queue, each request lacks a slot of its kind or (for the first one that
//    has a slot) its bytes exceed the free budget;
//  * slots and the budget are never overcommitted, and with completions every
//    request eventually starts.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "admission.h"

namespace {

struct Req {
    int id;
    bool fwd;
    size_t bytes;
};

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("check failed line %d: %s\n", __LINE__, #c);   \
            return 1;                                                   \
        }                                                               \
    } while (0)

int run(uint64_t seed, int slots, size_t budget, int steps) {
    std::mt19937_64 rng(seed);
    std::deque<Req *> queue;
    std::vector<Req *> active, all;
    int free_fwd = slots, free_inv = slots, next_id = 0, started_total = 0;
    size_t free_bytes = budget;
    int last_fwd = -1, last_inv = -1;
    for (int s = 0; s < steps || !queue.empty() || !active.empty(); ++s) {
        if (s < steps) {
            const int arrivals = (int)(rng() % 4);
            for (int a = 0; a < arrivals; ++a) {
                Req *r = new Req{next_id++, (rng() & 1) != 0, 1 + rng() % (budget / 3)};
                all.push_back(r);
                queue.push_back(r);
            }
        }
        const std::vector<Req *> before(queue.begin(), queue.end());
        std::vector<Req *> started;
        grav::admission_pass(
            queue, [](Req *r) { return r->fwd; },
            [&](bool fwd) { return (fwd ? free_fwd : free_inv) > 0; },
            [&](Req *r) {
                if (r->bytes > free_bytes) return false;
                free_bytes -= r->bytes;
                return true;
            },
            [&](Req *r, bool fwd) {
                (fwd ? free_fwd : free_inv) -= 1;
                started.push_back(r);
                active.push_back(r);
            });
        started_total += (int)started.size();
        CHECK(free_fwd >= 0 && free_inv >= 0 && free_fwd <= slots && free_inv <= slots);
        // order within kind, and the waiting queue keeps its relative order
        for (Req *r : started) {
            int &last = r->fwd ? last_fwd : last_inv;
            CHECK(r->id > last);
            last = r->id;
        }
        std::vector<Req *> waiting;
        for (Req *r : before)
            if (std::find(started.begin(), started.end(), r) == started.end()) waiting.push_back(r);
        CHECK(std::equal(waiting.begin(), waiting.end(), queue.begin(), queue.end()));
        // passing over: only inversions without a free inversion slot
        for (Req *w : waiting)
            for (Req *r : started)
                if (r->id > w->id) CHECK(!w->fwd && free_inv == 0);
        // the pass stopped where it had to
        for (Req *w : waiting) {
            const int free_slots = w->fwd ? free_fwd : free_inv;
            if (free_slots == 0) {
                if (w->fwd) break;      // nothing behind a slot-blocked forward may start
                continue;
            }
            CHECK(w->bytes > free_bytes);   // has a slot, so memory must be the reason
            break;
        }
        // completions
        for (size_t i = 0; i < active.size();) {
            if (rng() % 3 == 0) {
                Req *r = active[i];
                (r->fwd ? free_fwd : free_inv) += 1;
                free_bytes += r->bytes;
                active.erase(active.begin() + (long)i);
            } else {
                ++i;
            }
        }
        CHECK(s < steps + 100000);      // drains
    }
    CHECK(started_total == next_id && free_bytes == budget);
    CHECK(free_fwd == slots && free_inv == slots);
    for (Req *r : all) delete r;
    return 0;
}

}  // namespace

int main() {
    const int slot_counts[] = {1, 2, 5, 64};
    const size_t budgets[] = {1000, 100000};
    uint64_t seed = 1;
    for (int sc : slot_counts)
        for (size_t b : budgets)
            for (int k = 0; k < 20; ++k)
                if (run(seed++, sc, b, 400)) return 1;
    std::printf("ok\n");
    return 0;
}
