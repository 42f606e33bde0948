// lf2_batch_items.hpp -- passes of a batched Poisson solve and the order of
// the persistent kernel's work items (plain C++: the host batch code and the
// host model of the work queue both use it).
#pragma once
#include <stdint.h>

#include <array>
#include <vector>

#include "lf2_queue.hpp"

namespace lf2 {

// Passes of one field in a batched Poisson solve.
enum : int {
    BP_XF = 0,   // x r2c: rho -> W
    BP_YF = 1,   // y forward on W
    BP_Z = 2,    // z forward * -1/(N k^2) (+ binning) * z backward on W
    BP_YI = 3,   // y backward on W
    BP_XI = 4,   // x c2r: W -> phi
    BP_FIN = 5,  // power-spectrum finalize (one item)
    BP_COUNT = 6
};

// The pass an item of pass p waits for (-1: none): every pass needs the
// whole previous pass of its field (a y tile needs all x rows of its plane,
// a z tile every plane of its columns, ...); the finalize needs the z pass.
inline int batch_dep_pass(int p)
{
    switch (p) {
    case BP_YF: return BP_XF;
    case BP_Z: return BP_YF;
    case BP_YI: return BP_Z;
    case BP_XI: return BP_YI;
    case BP_FIN: return BP_Z;
    default: return -1;
    }
}

// Work items of a batch.  An item is up to `per_item` consecutive tiles of
// one pass of one field, sized by batch_chunks (the finalize is one item).  Queue q holds the
// items of the fields with
// queue_of[f] == q, pass by pass (x forward of every such field, then y, z,
// the finalizes, y backward, x backward), fields in order within a pass:
// every item comes after all the items it waits on, which is what the work
// queue needs.  The queues follow each other in the returned array:
// queue q is items [qstart[q], qstart[q] + qcount[q]).
// tiles[f][p] = tiles of pass p of field f (0: no item).  The counter of
// (f, p) is f * BP_COUNT + p and counts items.
// Item sizes of one pass of one field: per_item tiles while at least twice
// that many are left, then half of what is left (at least one), so that the
// pass's last items end close together and the next pass waits less.
inline std::vector<int> batch_chunks(int tiles, int per_item)
{
    std::vector<int> out;
    for (int left = tiles; left > 0;) {
        int n = left / 2;
        if (n > per_item) n = per_item;
        if (n < 1) n = 1;
        out.push_back(n);
        left -= n;
    }
    return out;
}
inline int batch_nitems(int tiles, int per_item)
{
    return (int)batch_chunks(tiles, per_item < 1 ? 1 : per_item).size();
}

inline std::vector<QItem> batch_items(const std::vector<std::array<int, BP_COUNT>> &tiles,
                                      int per_item, const std::vector<int> &queue_of, int nq,
                                      std::vector<uint32_t> &qstart, std::vector<uint32_t> &qcount)
{
    if (per_item < 1) per_item = 1;
    static const int order[BP_COUNT] = {BP_XF, BP_YF, BP_Z, BP_FIN, BP_YI, BP_XI};
    std::vector<QItem> items;
    const int nf = (int)tiles.size();
    qstart.assign(nq, 0);
    qcount.assign(nq, 0);
    for (int q = 0; q < nq; ++q) {
        qstart[q] = (uint32_t)items.size();
        for (int p : order)
            for (int f = 0; f < nf; ++f) {
                if (queue_of[f] != q) continue;
                const int dp = batch_dep_pass(p);
                const int need = dp < 0 ? 0 : batch_nitems(tiles[f][dp], per_item);
                int t = 0;
                for (int n : batch_chunks(tiles[f][p], per_item)) {
                    items.push_back(QItem{f, p, t, n, f * BP_COUNT + p,
                                          dp < 0 ? -1 : f * BP_COUNT + dp, need, 0});
                    t += n;
                }
            }
        qcount[q] = (uint32_t)items.size() - qstart[q];
    }
    return items;
}

// Fields to queues, longest processing time first: each field (largest
// `work` first) goes to the queue with the least work so far.
inline std::vector<int> balance_queues(const std::vector<double> &work, int nq)
{
    std::vector<int> order(work.size()), out(work.size(), 0);
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    for (size_t i = 1; i < order.size(); ++i)  // insertion sort, largest first, stable
        for (size_t j = i; j > 0 && work[order[j]] > work[order[j - 1]]; --j) {
            const int t = order[j];
            order[j] = order[j - 1];
            order[j - 1] = t;
        }
    std::vector<double> load(nq, 0.0);
    for (int f : order) {
        int best = 0;
        for (int q = 1; q < nq; ++q)
            if (load[q] < load[best]) best = q;
        out[f] = best;
        load[best] += work[f];
    }
    return out;
}

}  // namespace lf2
