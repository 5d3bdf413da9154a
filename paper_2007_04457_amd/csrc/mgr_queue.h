// Scheduling protocol of the persistent batched decomposition: one launch
// whose workgroups take work items from a queue in order and wait, before
// running an item, until every item it depends on has finished.  Internal;
// the same functions run on the device (mgr_batch.hip) and on host threads
// standing in for workgroups (mgr_batch_queue_check in mgr_api.cpp), so the
// protocol the kernel follows is the one the host check exercises.
//
// Items are numbered in an order where every item's dependencies come
// first: the items of one field's stage form a group, and a group depends on
// the previous group of the same field (its previous stage, or the last
// stage of its previous level step).  A workgroup
//   1. stops if the run was aborted, else takes the next index with one
//      atomic add (items beyond the last: stop);
//   2. waits until the completion counter of the item's dependency group
//      reaches that group's size, polling with relaxed agent-scope atomic
//      loads and sleeping between polls, then issues one acquire fence at
//      agent scope (the workgroup then sees the data those items wrote).
//      Polling with acquire loads instead would invalidate the caches on
//      every poll: on a device whose agent spans several L2 caches (one per
//      XCD) that stalls every working workgroup of the XCD;
//   3. runs the item, then adds one to its own group's counter with a
//      release at agent scope (its writes become visible first).
// Why it cannot deadlock: a workgroup takes an index only while it runs,
// indices are taken in increasing order, and an item only waits for items of
// smaller index.  The smallest unfinished index therefore belongs to a
// running workgroup that waits for nothing unfinished, and it finishes.
// Nothing here depends on how many workgroups are resident or on the grid
// size.  Every wait is bounded: after `limit` polls the waiter sets the run's
// abort flag and records the item in the error word; every workgroup checks
// the flag before taking an item and while it polls, so an aborted run ends
// within one poll bound of the first failed wait.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgr {

struct QueueTables {
    const int* grp;   // group of each item
    const int* dep;   // dependency group of each group (-1: none)
    const int* need;  // items in each group
    int total;        // items
};

struct QueueState {
    int* next;   // next index to hand out
    int* done;   // finished items per group
    int* abort;  // nonzero once a wait has timed out
    int* err;    // 1 + the item whose wait timed out first (0: none)
};

// Takes the next item and waits for its dependencies; -1 when the workgroup
// should stop (queue empty, run aborted, or this wait timed out).  On the
// device a whole wave runs it and every value involved is wave-uniform.
template <class Ops>
__host__ __device__ inline int queue_take(const QueueTables& t, const QueueState& s, unsigned limit, Ops ops)
{
    if (ops.load_relaxed(s.abort)) return -1;
    const int i = ops.fetch_add_relaxed(s.next, 1);
    if (i >= t.total) return -1;
    const int g = t.grp[i];
    const int dg = t.dep[g];
    if (dg < 0) return i;
    const int need = t.need[dg];
    unsigned polls = 0;
    while (ops.load_relaxed(&s.done[dg]) < need) {
        if (ops.load_relaxed(s.abort)) return -1;
        if (++polls > limit) {
            ops.cas_relaxed(s.err, 0, i + 1);
            ops.store_relaxed(s.abort, 1);
            return -1;
        }
        ops.pause();
    }
    ops.fence_acquire();
    return i;
}

// Marks item i finished, once every write of the item by every thread of
// the workgroup has completed (the caller waits for them), with a release at
// agent scope (on the device: a whole wave, one lane doing the atomic).
template <class Ops>
__host__ __device__ inline void queue_finish(const QueueTables& t, const QueueState& s, int i, Ops ops)
{
    ops.add_release(&s.done[t.grp[i]], 1);
}

}  // namespace mgr
