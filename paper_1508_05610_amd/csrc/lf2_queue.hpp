// lf2_queue.hpp -- the work queues of the persistent batch kernel: how a
// block claims work items, waits for the items an item depends on, and
// publishes its own completion.
//
// Written once over two policies so that the same code runs in the kernel
// (HIP atomics, __syncthreads, cache maintenance) and in a host model (std
// atomics, one std::thread per lane group of a block, std::barrier), where
// it is checked under ThreadSanitizer with fewer resident blocks than
// blocks.
//
// Protocol.  There are nq queues; a block serves one of them (the kernel
// picks the queue of the block's XCD, so that the producer and the consumer
// of every tile share one L2).  A queue's items sit in an array in which
// every item comes after all the items it depends on (the host orders them
// pass by pass).  A block takes the next item index of its queue from the
// queue's atomic ticket, so items are handed out in array order.  An item
// waits until the counter it depends on reaches the number of items it
// needs, runs, then adds one to its own counter.  Dependencies never cross
// queues.  No wait can block forever: every item an item waits on has a
// smaller index in the same queue, so it was handed out before, to a block
// that is running (a block only takes items while it runs); the unfinished
// item with the smallest index waits on nothing unfinished, so it
// completes, and so on upward -- for any number of resident blocks, one
// included, as long as each queue is served by at least one block.  Each
// wait is also bounded (spin_limit polls): past it the block sets bit 0 of
// the error word and goes on, and from then on no block waits, so the
// kernel ends within about one spin limit.  After its last claim each block
// counts itself out; the last one checks that every queue was emptied (bit
// 1 of the error word if not), then resets the tickets and the counters for
// the next run (the error word stays until the host reads and clears it).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define LF2_QFN __host__ __device__ __forceinline__
#else
#define LF2_QFN inline
#endif

namespace lf2 {

struct QItem {
    int32_t field;
    int32_t pass;
    int32_t tile;   // first tile of the item
    int32_t ntile;  // tiles tile .. tile + ntile - 1
    int32_t slot;   // counter this item adds one to when done
    int32_t dep;    // counter it waits on (-1: none)
    int32_t need;   // value of counter `dep` once everything it waits on is done
    int32_t pad;
};

// ctl[q].ticket: next item index of queue q; ctl[0].exited: blocks past
// their last claim; ctl[0].error: bit 0 a wait gave up, bit 1 a queue was
// left with unclaimed items.
struct QCtl {
    uint32_t ticket;
    uint32_t exited;
    uint32_t error;
    uint32_t pad;
};

// Atomics and memory-ordering policy A:
//   fetch_add_relaxed / fetch_add_acq_rel / fetch_or_relaxed, load_relaxed /
//   store_relaxed on uint32_t,
//   publish_add(p, v) the completion count of an item,
//   poll_load(p)      the count a wait polls,
//   wave_release()    every thread, after the item's stores,
//   leader_release()  the leader, after the block barrier, before publish_add,
//   leader_acquire()  the leader, after its wait,
//   wave_acquire()    every thread, after the block barrier that ends the wait,
//   pause()           between polls.
// A policy makes an item's stores visible to the readers of a published
// count either in publish_add / poll_load themselves (release / acquire) or
// through the wave and leader operations around them (then the two may be
// relaxed).
// B: one block: leader(), share(v) / shared() (one word the block shares),
// barrier().  work(item) runs the item on every thread; it may use the
// block's barrier, the same number of times on every thread.
// The leader is a group of threads that take the leader's branches together
// (one thread in the host model, the block's first wave on the GPU); A's
// operations, called by every thread of that group, act once and return the
// same result to each of them.
template <class A, class B, class Work>
LF2_QFN void run_queue(B &blk, QCtl *ctl, int q, int nq, uint32_t *done, int ndone,
                       const QItem *items, const uint32_t *qstart, const uint32_t *qcount,
                       uint32_t nblocks, uint32_t spin_limit, Work &&work)
{
    const QItem *mine = items + qstart[q];
    const uint32_t nitems = qcount[q];
    for (;;) {
        if (blk.leader()) blk.share(A::fetch_add_relaxed(&ctl[q].ticket, 1u));
        blk.barrier();
        const uint32_t t = blk.shared();
        blk.barrier();  // everyone has read t before the leader writes the next one
        if (t >= nitems) break;  // the same t on every thread: the whole block leaves
        const QItem it = mine[t];
        if (it.dep >= 0) {
            if (blk.leader()) {
                uint32_t polls = 0;
                while (A::poll_load(&done[it.dep]) < (uint32_t)it.need) {
                    // once any wait has given up, no block waits any more
                    if (++polls > spin_limit || A::load_relaxed(&ctl[0].error)) {
                        A::fetch_or_relaxed(&ctl[0].error, 1u);
                        break;
                    }
                    A::pause();
                }
                A::leader_acquire();
            }
            blk.barrier();
            A::wave_acquire();
        }
        work(it);
        A::wave_release();
        blk.barrier();
        if (blk.leader()) {
            A::leader_release();
            A::publish_add(&done[it.slot], 1u);
        }
    }
    if (blk.leader()) {
        if (A::fetch_add_acq_rel(&ctl[0].exited, 1u) == nblocks - 1) {
            // every other block has made its last claim and published its
            // last item: nothing reads or writes the queues any more
            for (int i = 0; i < nq; ++i) {
                if (A::load_relaxed(&ctl[i].ticket) < qcount[i]) A::fetch_or_relaxed(&ctl[0].error, 2u);
                A::store_relaxed(&ctl[i].ticket, 0u);
            }
            for (int i = 0; i < ndone; ++i) A::store_relaxed(&done[i], 0u);
            A::store_relaxed(&ctl[0].exited, 0u);
        }
    }
}

}  // namespace lf2
