"""The persistent batch's scheduling protocol on host threads (no GPU).

mgr_batch_queue_check builds a batch's work items, waves, queues (one per
XCD on the device; every field in one queue) and dependency groups on the
host and runs the very queue functions the persistent kernel runs
(mgr_queue.h) on host threads standing in for workgroups, thread t serving
queue t mod nqueues.  These tests pin what the kernel relies on: every item
runs exactly once and only after every item it depends on has finished,
whatever the number of workers, queues and the timing; a worker that never
finishes its item makes the bounded waits behind it run out, the run aborts,
names the position whose wait ran out, and every worker ends, with nothing
started that depended on the stalled item.
"""
import pytest

import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import synth

WORKLOAD = [s for s, _ in synth.batched_shapes()]
MIXED = [(33, 17, 65), (65, 65, 65), (129, 129), (17, 9, 33), (257,), (9, 9, 9), (513, 257), (5, 5, 9),
         (129, 33, 65), (1025, 9), (16385,), (5, 5, 1025)]


@pytest.mark.parametrize("nthreads,nqueues", [(1, 1), (2, 1), (7, 1), (2, 2), (8, 8), (32, 8), (256, 8), (48, 16)])
@pytest.mark.parametrize("chunk", [8, 32])
def test_every_item_runs_once_after_its_dependencies(nthreads, nqueues, chunk):
    ran, early, err, untaken = mgr.batch_queue_check(WORKLOAD, chunk=chunk, nthreads=nthreads, nqueues=nqueues,
                                                     seed=nthreads)
    assert (early, err, untaken) == (0, 0, 0)
    assert ran > 80000  # the 96-field workload's items
    # the same items whatever the number of queues
    assert ran == mgr.batch_queue_check(WORKLOAD, chunk=chunk, nthreads=4, nqueues=1)[0]


@pytest.mark.parametrize("seed", range(4))
def test_mixed_shapes_and_types(seed):
    for dt in (mgr.MGR_F32, mgr.MGR_F64):
        ran, early, err, untaken = mgr.batch_queue_check(MIXED, dtype_code=dt, nthreads=12, nqueues=4, seed=seed)
        assert (early, err, untaken) == (0, 0, 0) and ran > 0


def test_queue_without_workers_is_left_untaken():
    """A queue that no worker serves keeps its items (the device deals
    workgroups to every XCD, so there each queue has workers)."""
    total = mgr.batch_queue_check(WORKLOAD, nthreads=8, nqueues=8)[0]
    ran, early, err, untaken = mgr.batch_queue_check(WORKLOAD, nthreads=7, nqueues=8)
    assert early == 0 and err == 0 and untaken > 0 and ran + untaken == total


@pytest.mark.parametrize("frac", [0.0, 0.3, 0.7])
def test_stalled_workgroup_aborts_the_run(frac):
    total = mgr.batch_queue_check(WORKLOAD, nthreads=8)[0]
    stall = int(frac * (total - 1))
    # a bound far above any legitimate wait here (host polls take well
    # under a microsecond): only waits on the stalled item run out
    ran, early, err, untaken = mgr.batch_queue_check(WORKLOAD, nthreads=16, poll_limit=2_000_000, stall_item=stall,
                                                     seed=11)
    assert early == 0          # nothing started before its dependencies
    assert err > stall + 1     # a later position's wait ran out (err = 1 + that position)
    assert ran <= total - 1 and ran + untaken < total


def test_stall_of_an_item_nothing_depends_on_finishes_normally():
    total = mgr.batch_queue_check(WORKLOAD, nthreads=8)[0]
    ran, early, err, untaken = mgr.batch_queue_check(WORKLOAD, nthreads=8, poll_limit=2_000_000, stall_item=total - 1)
    assert (ran, early, err, untaken) == (total - 1, 0, 0, 0)
