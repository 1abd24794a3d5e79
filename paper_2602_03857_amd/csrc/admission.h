// One admission pass of the server's scheduler over its queue of waiting
// requests, in arrival order.  Plain C++ (no HIP), so the policy is also
// checked on the host under the address and undefined-behaviour sanitizers.
//
// Policy: inversions start in arrival order while an inversion slot is free;
// forward requests start in arrival order on their own slots and may pass
// inversions that wait only for an inversion slot; device memory is granted
// strictly in arrival order (the first request that does not fit ends the
// pass, so nothing behind it starts).
#pragma once

namespace grav {

// queue: a sequence container (begin, end, erase) of waiting requests, front =
// oldest.  is_forward(q): request kind.  has_slot(forward): a slot of that
// kind is free.  try_alloc(q): reserves the request's device memory, false if
// it does not fit.  start(q, forward): takes a slot and starts the request.
// Started requests are removed from the queue; the rest keep their order.
template <class Queue, class IsForward, class HasSlot, class TryAlloc, class Start>
void admission_pass(Queue &queue, IsForward is_forward, HasSlot has_slot, TryAlloc try_alloc,
                    Start start) {
    bool inv_blocked = false;
    for (auto it = queue.begin(); it != queue.end();) {
        const bool fwd = is_forward(*it);
        if (!has_slot(fwd)) {
            if (fwd) break;           // forward requests keep their order
            inv_blocked = true;       // forward requests behind it may pass
            ++it;
            continue;
        }
        if (!fwd && inv_blocked) {    // inversions keep their order
            ++it;
            continue;
        }
        if (!try_alloc(*it)) break;   // memory: strict arrival order
        start(*it, fwd);
        it = queue.erase(it);
    }
}

}  // namespace grav
