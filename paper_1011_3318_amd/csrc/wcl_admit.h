// Admission policy of the serving loop, as a pure function of the server's
// memory state, so that it can be checked on the host without a device.
//
// A slot keeps the workspace of its last solves; its named buffers only grow
// (a buffer is reallocated only when a request needs it larger), and freeing
// device memory stalls every stream of the device, so workspaces are kept
// whenever the budget allows.  A request reuses an idle slot's workspace at
// no charge when it was built for the same lattice and solver parameters;
// otherwise it takes the idle slot holding the most memory and is charged
// its full estimate (an upper bound of that workspace's growth).  Only when
// that does not fit the budget is the chosen slot's workspace released, and
// then the other idle slots' too.  With no solve running, everything but the
// resident fields can be released, so a request that fits the budget next
// to the resident fields (which wcl_submit checks) is always admitted: the
// queue cannot stall.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

struct AdmitSlot {
    bool busy;
    size_t held;     // bytes the slot's workspace holds
    uint64_t key;    // what the workspace was built for (0 = nothing)
};

struct AdmitDecision {
    int slot = -1;               // -1: the request waits
    bool release_slot = false;   // free the chosen slot's workspace first
    bool release_idle = false;   // free the workspaces of all other idle slots first
    size_t charge = 0;           // bytes reserved for the solve's allocations
};

// resident: resident gauge/clover fields; reserved: bytes charged to the
// running solves; need / key: the request's workspace estimate and key.
inline AdmitDecision admit_decide(const std::vector<AdmitSlot>& slots, size_t budget, size_t resident,
                                  size_t reserved, size_t need, uint64_t key) {
    AdmitDecision d;
    size_t held_all = 0, held_busy = 0;
    int reuse = -1, other = -1;
    for (size_t k = 0; k < slots.size(); ++k) {
        held_all += slots[k].held;
        if (slots[k].busy) {
            held_busy += slots[k].held;
            continue;
        }
        if (reuse < 0 && slots[k].key == key && key != 0) reuse = (int)k;
        // the idle slot holding the most memory is the one to release
        if (other < 0 || slots[k].held > slots[other].held) other = (int)k;
    }
    if (other < 0) return d;   // no idle slot
    if (reuse >= 0 && resident + held_all + reserved <= budget) {
        d.slot = reuse;
        return d;
    }
    if (resident + held_all + reserved + need <= budget) {   // keep every workspace
        d.slot = other;
        d.charge = need;
        return d;
    }
    if (resident + held_all - slots[other].held + reserved + need <= budget) {
        d.slot = other;
        d.release_slot = true;
        d.charge = need;
        return d;
    }
    if (resident + held_busy + reserved + need <= budget) {
        d.slot = other;
        d.release_slot = true;
        d.release_idle = true;
        d.charge = need;
        return d;
    }
    return d;   // waits for a running solve to finish
}
