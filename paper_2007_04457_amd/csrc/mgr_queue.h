// Scheduling protocol of the persistent batched decomposition: one launch
// whose workgroups take work items from queues in order and wait, before
// running an item, until every item it depends on has finished.  Internal;
// the same functions run on the device (mgr_batch.hip) and on host threads
// standing in for workgroups (mgr_batch_queue_check in mgr_api.cpp), so the
// protocol the kernel follows is the one the host check exercises.
//
// There is one queue per XCD (an accelerator die with its own L2 cache), and
// every field's items are in one queue: a workgroup takes items only from
// the queue of the XCD it runs on, so an item and every item it depends on
// run under one L2, and making an item's results visible to the items that
// depend on it never needs the L2 written back to memory (on a device whose
// agent spans several L2 caches each such write-back stalls the whole XCD).
// Within a queue, positions are numbered in an order where every item's
// dependencies come first: the items of one field's stage form a group, and
// a group depends on the previous group of the same field (its previous
// stage, or the last stage of its previous level step).  A workgroup
//   1. stops if the run was aborted, else takes the next position of its
//      queue with one atomic add (positions beyond the queue's last: stop);
//   2. waits until the completion counter of the position's dependency group
//      reaches that group's size, polling with relaxed loads and sleeping
//      between polls, then invalidates its caches' clean lines (its CU's L1
//      may hold lines read before the producers wrote them; the producers'
//      data is in the shared L2, dirty lines are kept).  A workgroup that has
//      already waited for the same dependency group skips both: the group
//      was complete then, and the items of one stage read only the data of
//      earlier stages and their own parts of the stage's outputs, so no line
//      it has read since can have been changed under it by another item;
//   3. runs the item, waits until every store of the item has reached the
//      L2 (all threads), and adds one to its group's counter.
// Why it cannot deadlock: a workgroup takes a position only while it runs,
// positions of a queue are taken in increasing order, and an item only waits
// for items of smaller position in the same queue.  In every queue the
// smallest unfinished position therefore belongs to a running workgroup that
// waits for nothing unfinished, and it finishes; every XCD runs workgroups of
// the launch until its queue is empty.  Nothing here depends on how many
// workgroups are resident or on the grid size.  Every wait is bounded: after
// `limit` polls the waiter sets the run's abort flag and records the position
// in the error word; every workgroup checks the flag before taking a
// position and while it polls, so an aborted run ends within one poll bound
// of the first failed wait.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgr {

constexpr int kMaxQueues = 16;

struct QueueTables {
    const int* grp;    // group of each position
    const int* dep;    // dependency group of each group (-1: none)
    const int* need;   // items in each group
    const int* order;  // item at each position
    int nq;            // queues
    int start[kMaxQueues + 1];  // positions of queue q: [start[q], start[q + 1])
};

// Queue words: abort, err, next[kMaxQueues], done[groups] (kQueueWordsFixed
// words before the counters).
constexpr int kQueueWordsFixed = 2 + kMaxQueues;
struct QueueState {
    int* abort;  // nonzero once a wait has timed out
    int* err;    // 1 + the position whose wait timed out first (0: none)
    int* next;   // next position to hand out, per queue (relative to its start)
    int* done;   // finished items per group
};

// Takes the next position of queue q and waits for its dependencies; -1
// when the workgroup should stop (queue empty, run aborted, or this wait
// timed out).  last_dg: the dependency group this workgroup last waited for
// (-1 at first; updated here).  On the device a whole wave runs it and every
// value involved is wave-uniform.
template <class Ops>
__host__ __device__ inline int queue_take(const QueueTables& t, const QueueState& s, int q, unsigned limit,
                                          int& last_dg, Ops ops)
{
    if (ops.load_relaxed(s.abort)) return -1;
    const int j = ops.fetch_add_relaxed(&s.next[q], 1);
    if (j >= t.start[q + 1] - t.start[q]) return -1;
    const int i = t.start[q] + j;
    const int g = t.grp[i];
    const int dg = t.dep[g];
    if (dg < 0 || dg == last_dg) return i;
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
    last_dg = dg;
    return i;
}

// Marks position i finished, once every store of the item by every thread
// of the workgroup has completed (the caller waits for them); on the device
// a whole wave runs it, one lane doing the atomic.
template <class Ops>
__host__ __device__ inline void queue_finish(const QueueTables& t, const QueueState& s, int i, Ops ops)
{
    ops.add_release(&s.done[t.grp[i]], 1);
}

}  // namespace mgr
