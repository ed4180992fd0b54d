// Host-only checks of the serving loop's admission policy (admit_decide).
// Built with g++ by tests/test_admission.py; prints one line per check and
// exits non-zero on the first failure.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "wcl_admit.h"

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                          \
        }                                                          \
    } while (0)

int main() {
    const size_t MB = 1 << 20;
    // no idle slot: wait
    {
        std::vector<AdmitSlot> s = {{true, 10 * MB, 7}};
        CHECK(admit_decide(s, 100 * MB, 0, 10 * MB, 5 * MB, 7).slot == -1);
        std::printf("ok no-idle-slot\n");
    }
    // same lattice and parameters: the idle slot's workspace is reused at no charge
    {
        std::vector<AdmitSlot> s = {{false, 30 * MB, 5}, {false, 10 * MB, 7}};
        AdmitDecision d = admit_decide(s, 100 * MB, 20 * MB, 0, 30 * MB, 7);
        CHECK(d.slot == 1 && !d.release_slot && !d.release_idle && d.charge == 0);
        std::printf("ok reuse\n");
    }
    // another lattice, budget to spare: the idle workspace holding the most is
    // kept (it grows by at most the charge), nothing is released
    {
        std::vector<AdmitSlot> s = {{false, 30 * MB, 5}, {false, 10 * MB, 7}};
        AdmitDecision d = admit_decide(s, 200 * MB, 20 * MB, 0, 50 * MB, 9);
        CHECK(d.slot == 0 && !d.release_slot && !d.release_idle && d.charge == 50 * MB);
        std::printf("ok keep\n");
    }
    // the stall that a growth-only charge allowed: two idle slots hold small
    // workspaces, a large request of another lattice arrives, nothing runs
    {
        std::vector<AdmitSlot> s = {{false, 40 * MB, 3}, {false, 40 * MB, 3}};
        AdmitDecision d = admit_decide(s, 100 * MB, 10 * MB, 0, 85 * MB, 9);
        CHECK(d.slot >= 0 && d.release_slot && d.release_idle && d.charge == 85 * MB);
        std::printf("ok idle-release\n");
    }
    // one solve running: the request waits until it fits beside it
    {
        std::vector<AdmitSlot> s = {{true, 0, 3}, {false, 40 * MB, 3}};
        CHECK(admit_decide(s, 100 * MB, 10 * MB, 60 * MB, 50 * MB, 9).slot == -1);
        AdmitDecision d = admit_decide(s, 100 * MB, 10 * MB, 30 * MB, 50 * MB, 9);
        CHECK(d.slot == 1 && d.release_slot && d.charge == 50 * MB);
        std::printf("ok wait-for-running\n");
    }
    // Random streams of requests (4 lattices, 2 parameter sets each) on 1-4
    // slots under budgets from tight to loose: every request is admitted, the
    // memory in use never exceeds the budget, and the queue never stalls
    // while nothing runs.
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 400; ++trial) {
        const int nslots = 1 + (int)(rng() % 4);
        const size_t resident = (5 + rng() % 20) * MB;
        const size_t sizes[4] = {2 * MB, 9 * MB, 30 * MB, 70 * MB};
        const size_t budget = resident + sizes[3] + (rng() % 3) * 40 * MB;
        struct Req {
            size_t need;
            uint64_t key;
            int left;   // remaining work units once admitted
        };
        std::deque<Req> queue;
        for (int k = 0; k < 200; ++k) {
            int lat = (int)(rng() % 4);
            queue.push_back({sizes[lat], (uint64_t)(1 + 2 * lat + rng() % 2), 1 + (int)(rng() % 5)});
        }
        std::vector<AdmitSlot> slots(nslots, AdmitSlot{false, 0, 0});
        std::vector<Req> running(nslots);
        std::vector<size_t> charged(nslots, 0);
        size_t reserved = 0;
        int done = 0, ticks = 0;
        while (done < 200) {
            CHECK(++ticks < 100000);
            // admit as long as the policy allows
            for (;;) {
                if (queue.empty()) break;
                AdmitDecision d = admit_decide(slots, budget, resident, reserved, queue.front().need,
                                               queue.front().key);
                if (d.slot < 0) break;
                if (d.release_idle)
                    for (int k = 0; k < nslots; ++k)
                        if (!slots[k].busy && k != d.slot) slots[k] = AdmitSlot{false, 0, 0};
                if (d.release_slot) slots[d.slot] = AdmitSlot{false, 0, 0};
                slots[d.slot].busy = true;
                slots[d.slot].key = queue.front().key;
                running[d.slot] = queue.front();
                charged[d.slot] = d.charge;
                reserved += d.charge;
                queue.pop_front();
            }
            size_t held = 0;
            bool any_busy = false;
            for (int k = 0; k < nslots; ++k) {
                held += slots[k].held;
                any_busy = any_busy || slots[k].busy;
            }
            CHECK(resident + held + reserved <= budget);
            CHECK(any_busy || queue.empty());   // nothing runs only when nothing waits
            // one unit of work on every running solve; a charged solve's
            // workspace grows by at most its charge (worst case modelled)
            for (int k = 0; k < nslots; ++k) {
                if (!slots[k].busy) continue;
                if (--running[k].left > 0) continue;
                reserved -= charged[k];
                slots[k].held += charged[k];
                slots[k].busy = false;
                ++done;
            }
        }
    }
    std::printf("ok random-streams\n");
    return 0;
}
