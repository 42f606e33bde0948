// Host model of the persistent batch kernel's work queue (lf2_queue.hpp):
// the kernel's own claim / wait / publish code, run by std::threads.
//
// A block is W threads sharing one std::barrier, as a workgroup shares
// __syncthreads.  Blocks start in index order but only R of them may be
// resident at once (a block takes a residency slot before it starts and
// gives it back when it ends), as the GPU keeps launching blocks while
// others are still running.  Items stamp their tile of a per-(field, pass)
// array with plain stores, and an item checks, with plain loads, that every
// tile of the pass it depends on is stamped: under ThreadSanitizer a missing
// happens-before edge in the protocol shows up as a data race, and a wrong
// order as a failed check.
//
// Fields are spread over nq queues as the batch code spreads them over the
// XCDs (balance_queues), and block b serves queue b mod nq, as blocks go to
// the XCDs in turn.
//
// usage: queue_model <mode> <blocks> <resident> <threads/block> <seed> <fields> [queues]
//   mode  ticket  : the shipped protocol (items in dependency order)
//         static  : item = block + k * blocks (no ticket, one queue): blocks
//                   wait on items of blocks that are not resident yet
//         reverse : the ticket protocol over an item order that is not a
//                   dependency order
//         starved : the ticket protocol with one queue that no block serves
// Prints one line "mode=... items=... processed=... errors=... reset=..."
// and exits 0 when every item ran once, no wait gave up, every check passed
// and the queues were reset; 1 otherwise.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <barrier>
#include <condition_variable>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1508_05610_amd/csrc/lf2_batch_items.hpp"
#include "../../paper_1508_05610_amd/csrc/lf2_queue.hpp"

using namespace lf2;

struct HostAtomics {
    static uint32_t fetch_add_relaxed(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
    // the host model orders an item's stores through the counts themselves
    static uint32_t publish_add(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELEASE); }
    static uint32_t fetch_add_acq_rel(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
    static uint32_t fetch_or_relaxed(uint32_t *p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
    static uint32_t load_relaxed(const uint32_t *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    static uint32_t poll_load(const uint32_t *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
    static void store_relaxed(uint32_t *p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    // The block barrier (std::barrier) already orders the threads of a
    // block; the kernel's per-thread agent-scope fences have no host analogue.
    static void wave_release() {}
    static void leader_release() {}
    static void leader_acquire() {}
    static void wave_acquire() {}
    static void pause() { std::this_thread::yield(); }
};

struct HostBlock {
    std::barrier<> *bar;
    uint32_t *word;
    int lane;
    bool leader() const { return lane == 0; }
    void share(uint32_t v) { *word = v; }
    uint32_t shared() const { return *word; }
    void barrier() { bar->arrive_and_wait(); }
};

// residency slots, handed out in block order
struct Slots {
    std::mutex mu;
    std::condition_variable cv;
    int free_slots;
    int next = 0;  // next block allowed to start
    void acquire(int b)
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return next == b && free_slots > 0; });
        --free_slots;
        ++next;
        cv.notify_all();
    }
    void release()
    {
        std::lock_guard<std::mutex> lk(mu);
        ++free_slots;
        cv.notify_all();
    }
};

int main(int argc, char **argv)
{
    if (argc < 7) {
        fprintf(stderr, "usage: %s mode blocks resident threads seed fields\n", argv[0]);
        return 2;
    }
    const std::string mode = argv[1];
    const int G = atoi(argv[2]), R = atoi(argv[3]), W = atoi(argv[4]);
    const unsigned seed = (unsigned)atoi(argv[5]);
    const int F = atoi(argv[6]);
    int NQ = argc > 7 ? atoi(argv[7]) : 1;
    if (mode == "static") NQ = 1;
    std::mt19937 rng(seed);
    // tiles per (field, pass): x passes and y / z passes of uneven fields
    std::vector<std::array<int, BP_COUNT>> tiles(F);
    for (auto &t : tiles) {
        std::uniform_int_distribution<int> d(1, 12);
        t[BP_XF] = t[BP_XI] = d(rng);
        t[BP_YF] = t[BP_YI] = d(rng);
        t[BP_Z] = d(rng);
        t[BP_FIN] = 1;
    }
    std::vector<double> fwork(F);
    for (int f = 0; f < F; ++f) fwork[f] = tiles[f][BP_XF] + tiles[f][BP_YF] + tiles[f][BP_Z];
    const std::vector<int> queue_of = balance_queues(fwork, NQ);
    std::vector<uint32_t> qstart, qcount;
    // 1 to 3 tiles per item
    const int per_item = 1 + (int)(seed % 3);
    std::vector<QItem> items = batch_items(tiles, per_item, queue_of, NQ, qstart, qcount);
    if (mode == "reverse") {
        // within every queue, a late-pass item first: it waits on items that come after it
        for (int q = 0; q < NQ; ++q)
            std::reverse(items.begin() + qstart[q], items.begin() + qstart[q] + qcount[q]);
    }
    const int ndone = F * BP_COUNT;
    std::vector<uint32_t> done(ndone, 0);
    std::vector<QCtl> ctls(NQ, QCtl{0, 0, 0, 0});
    QCtl &ctl = ctls[0];
    // per-(field, pass) tile stamps, plain memory
    std::vector<std::vector<int>> stamp(ndone);
    for (int f = 0; f < F; ++f)
        for (int p = 0; p < BP_COUNT; ++p) stamp[f * BP_COUNT + p].assign(tiles[f][p], 0);
    // runs of each (counter, tile): every item exactly once
    std::vector<std::vector<std::atomic<int>>> runs(ndone);
    for (int i = 0; i < ndone; ++i) runs[i] = std::vector<std::atomic<int>>(stamp[i].size());
    std::atomic<int> bad{0};
    // waits of the ticket protocol always end (a poll yields the core, so an
    // oversubscribed host can stretch one a long way); the deadlocking
    // orders end only through the limit
    const uint32_t spin_limit = mode == "ticket" ? 50000000u : 200000u;

    auto work = [&](const QItem &it, int lane, std::barrier<> &bar) {
        // every lane checks a share of the dependency's tiles, then the
        // leader stamps the item's tile (after a barrier, like a tile's
        // store phase)
        if (it.dep >= 0) {
            const auto &src = stamp[it.dep];
            for (size_t i = lane; i < src.size(); i += W)
                if (src[i] != 1) bad.fetch_add(1);
        }
        bar.arrive_and_wait();
        if (lane == 0) {
            for (int t = it.tile; t < it.tile + it.ntile; ++t) {
                stamp[it.slot][t] = 1;
                runs[it.slot][t].fetch_add(1);
            }
        }
    };

    Slots slots;
    slots.free_slots = R;
    std::vector<std::thread> th;
    for (int b = 0; b < G; ++b) {
        th.emplace_back([&, b] {
            slots.acquire(b);
            std::barrier<> bar(W);
            uint32_t word = 0;
            std::vector<std::thread> lanes;
            for (int l = 0; l < W; ++l) {
                lanes.emplace_back([&, l] {
                    HostBlock blk{&bar, &word, l};
                    if (mode == "static") {
                        // fixed assignment, same wait / publish code
                        for (size_t t = b; t < items.size(); t += G) {
                            const QItem &it = items[t];
                            if (it.dep >= 0 && blk.leader()) {
                                uint32_t polls = 0;
                                while (HostAtomics::poll_load(&done[it.dep]) < (uint32_t)it.need) {
                                    if (++polls > spin_limit || HostAtomics::load_relaxed(&ctl.error)) {
                                        HostAtomics::fetch_or_relaxed(&ctl.error, 1u);
                                        break;
                                    }
                                    HostAtomics::pause();
                                }
                            }
                            blk.barrier();
                            work(it, l, bar);
                            blk.barrier();
                            if (blk.leader()) HostAtomics::publish_add(&done[it.slot], 1u);
                        }
                    } else {
                        // block b serves queue b mod NQ; "starved": no block serves the last queue
                        int q = b % NQ;
                        if (mode == "starved" && NQ > 1 && q == NQ - 1) q = 0;
                        run_queue<HostAtomics>(blk, ctls.data(), q, NQ, done.data(), ndone,
                                               items.data(), qstart.data(), qcount.data(),
                                               (uint32_t)G, spin_limit,
                                               [&](const QItem &it) { work(it, l, bar); });
                    }
                });
            }
            for (auto &t : lanes) t.join();
            slots.release();
        });
    }
    for (auto &t : th) t.join();
    int once = 0;
    for (auto &rs : runs)
        for (auto &r : rs) once += r.load() == 1;
    bool reset = ctl.exited == 0;
    for (auto &c : ctls) reset = reset && c.ticket == 0;
    for (uint32_t d : done) reset = reset && d == 0;
    int ntiles = 0;
    for (auto &rs : runs) ntiles += (int)rs.size();
    const bool ok = once == ntiles && ctl.error == 0 && bad.load() == 0 && reset;
    printf("mode=%s blocks=%d resident=%d threads=%d fields=%d queues=%d items=%zu "
           "tiles_processed_once=%d/%d errors=%u bad_checks=%d reset=%d ok=%d\n",
           mode.c_str(), G, R, W, F, NQ, items.size(), once, ntiles, ctl.error, bad.load(),
           reset ? 1 : 0, ok ? 1 : 0);
    return ok ? 0 : 1;
}
