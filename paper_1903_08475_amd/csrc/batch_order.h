// Queue order of the work items of a batched solve (plain C++, no HIP: the
// CPU tests compile it on its own).
//
// Every field of a batch goes through its stages in order (input split,
// moment contraction, radial scans, expansion: Sec. 4.3 steps 2, 4 and 5);
// an item of stage s of field f may start once every item of stage s-1 of
// field f has finished.  The persistent kernel's blocks take items from one
// queue in order; this header fixes that order by a list-scheduling
// simulation on the kernel's block count, with estimated item costs.
#pragma once

#include <algorithm>
#include <vector>

#include "ksplit.h"

namespace mpg {

// One work item: field f, stage st (0 .. n_stages-1), its index within
// (f, st), and an estimated cost (any time unit).
struct OrderItem {
    int f, st, idx;
    double cost;
};

// Returns the indices of `items` in queue order.  Simulation: `workers`
// workers; whenever one is free, it starts, among the items whose field's
// previous stage has finished, the one with the earliest latest start: the
// field's due time minus the item's remaining chain (its cost plus the
// costliest item of every later stage of its field).  Due times: the
// fields in increasing order of work get due times from half to all of an
// even share of the whole batch's work, in proportion to their cumulative
// work (never earlier than their own chain), so small fields finish early
// and the longest chains still start in time.  If no item is ready, the worker waits for
// the earliest stage release.  The queue is the order of the simulated
// starts, so every item comes after every item of its field's previous
// stage: a kernel whose blocks take items in this order only ever waits
// for items that running blocks have taken.
inline std::vector<int> order_items(const std::vector<OrderItem> &items, int n_fields, int n_stages, int workers) {
    const int ns = n_fields * n_stages;
    std::vector<std::vector<int>> stage(ns);  // item indices of (f, st), costliest first
    for (int i = 0; i < (int)items.size(); ++i) stage[items[i].f * n_stages + items[i].st].push_back(i);
    std::vector<double> maxc(ns, 0.0), tail(ns, 0.0);
    for (int s = 0; s < ns; ++s) {
        std::stable_sort(stage[s].begin(), stage[s].end(),
                         [&](int a, int b) { return items[a].cost > items[b].cost; });
        for (int i : stage[s]) maxc[s] = std::max(maxc[s], items[i].cost);
    }
    for (int f = 0; f < n_fields; ++f)
        for (int st = n_stages - 2; st >= 0; --st)
            tail[f * n_stages + st] = tail[f * n_stages + st + 1] + maxc[f * n_stages + st + 1];
    // due times
    std::vector<double> work(n_fields, 0.0), due(n_fields, 0.0);
    double total = 0.0;
    for (const OrderItem &it : items) {
        work[it.f] += it.cost;
        total += it.cost;
    }
    std::vector<int> rank(n_fields);
    for (int f = 0; f < n_fields; ++f) rank[f] = f;
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return work[a] < work[b]; });
    const double span = total / std::max(workers, 1);
    double cum = 0.0;
    for (int f : rank) {
        cum += work[f];
        const double chain = maxc[f * n_stages] + tail[f * n_stages];
        due[f] = std::max(span * (0.5 + 0.5 * cum / (total > 0.0 ? total : 1.0)), chain);
    }
    // release time of each stage (< 0: not yet known), items taken so far,
    // latest simulated finish of each stage's items
    std::vector<double> release(ns, -1.0), fin(ns, 0.0);
    std::vector<int> taken(ns, 0);
    for (int f = 0; f < n_fields; ++f) {
        // the first stage with items is released at once; empty stages pass
        int st = 0;
        while (st < n_stages && stage[f * n_stages + st].empty()) ++st;
        if (st < n_stages) release[f * n_stages + st] = 0.0;
    }
    std::vector<double> free_at(std::max(workers, 1), 0.0);
    std::vector<int> out;
    out.reserve(items.size());
    while (out.size() < items.size()) {
        const int w = (int)(std::min_element(free_at.begin(), free_at.end()) - free_at.begin());
        double t = free_at[w];
        // earliest release among stages with items left, if none is ready by t
        int best = -1;
        double best_p = 0.0, first_rel = -1.0;
        for (int s = 0; s < ns; ++s) {
            if (release[s] < 0.0 || taken[s] >= (int)stage[s].size()) continue;
            if (first_rel < 0.0 || release[s] < first_rel) first_rel = release[s];
        }
        if (first_rel < 0.0) break;  // cannot happen: some stage is always released
        if (first_rel > t) t = first_rel;
        for (int s = 0; s < ns; ++s) {
            if (release[s] < 0.0 || release[s] > t || taken[s] >= (int)stage[s].size()) continue;
            const int i = stage[s][taken[s]];
            const double p = due[s / n_stages] - (items[i].cost + tail[s]);  // latest start
            if (best < 0 || p < best_p) {
                best_p = p;
                best = s;
            }
        }
        const int i = stage[best][taken[best]++];
        out.push_back(i);
        free_at[w] = t + items[i].cost;
        fin[best] = std::max(fin[best], free_at[w]);
        if (taken[best] == (int)stage[best].size()) {
            // the next non-empty stage of the field is released when this one ends
            const int f = best / n_stages;
            int st = best % n_stages + 1;
            while (st < n_stages && stage[f * n_stages + st].empty()) ++st;
            if (st < n_stages) release[f * n_stages + st] = fin[best];
        }
    }
    return out;
}

}  // namespace mpg

namespace mpg {

// Work of one field of a split-form batch, in the units of the fused
// persistent kernel (tiles of 128, K slabs of 32 cells or moments).  A
// contraction block is 128 rows x 256 columns (two column tiles, one row
// tile) or 256 x 128 (one column tile, two row tiles), as the field's plan
// chose; its row and column units count blocks of that shape.
struct FieldShape {
    int split_units;            // input split: units of 2048 16-byte chunks
    int rows1;                  // moment contraction: row units
    int units_e, units_o;       // column units of the even / odd block
    int six_e, six_o;           // leading column units of each block with six products
    int kang;                   // moment contraction: K (angular cells, a multiple of 128)
    int splitk_min, splitk_max; // K splits: at least, at most (its work space)
    int scan_blocks, n_r;       // radial scans: column blocks of 64, shells
    int chunks;                 // radial scans: shell chunks per column
    int rows2, cols2;           // expansion: row units and angular units
    int k2_three, k2_six;       // expansion: K slabs with three / six products
};

// A queue entry of the fused kernel: field f, stage st (0 input split,
// 1 moments, 2 radial scans, 3 expansion) and the stage's block
// coordinates: split (first unit, units), moments (column unit, row unit,
// K split), scans (column block), expansion (row unit, first angular unit,
// angular units).
struct FusedItem {
    int f, st, a, b, c;
};

constexpr int kFusedStages = 4;
// Item sizes: input-split units per item, and expansion blocks (angular
// units of one row unit) per item.  Larger items pay the end of an item
// (waiting for its stores, counting it) less often.
constexpr int kSplitUnitsPerItem = 16;
constexpr int kExpansionUnitsPerItem = 2;

// Estimated item costs (microseconds on one CU of the target), from the
// fused kernel's own item times on the batching workload: per split unit,
// per K slab of a moment block (plus its start and end), per shell chunk
// step of a scan (eight thread rows take the chunks in turns), and per K
// slab of an expansion block plus its fixed cost (ring starts of its four
// runs, its output stores).  sk: K splits.
inline double fused_cost(const FieldShape &s, int sk, int st, int a, int b) {
    switch (st) {
        case 0: return 11.0 * b;
        case 1: {
            const bool six = a < s.units_e ? a < s.six_e : a - s.units_e < s.six_o;
            return 4.0 + ksplit_chunk(s.kang, sk, 32) / 32 * (six ? 2.75 : 1.85);
        }
        case 2: {
            const int ch = std::max(s.chunks, 1);
            return 1.75 * ((ch + 7) / 8) * ((s.n_r + ch - 1) / ch) * (1.0 + sk / 3.0);
        }
        default: return 18.0 + 1.66 * s.k2_three + 2.5 * s.k2_six;
    }
}

// Longest moment-contraction item the batch aims for (microseconds): a
// field whose K walk is longer is split further (up to its work space), so
// that no single item holds its field's later stages back for long.
constexpr double kMaxMomentItem = 500.0;

// K splits of a field in the fused batch
inline int fused_splitk(const FieldShape &s) {
    const double walk = s.kang / 32 * 2.4;
    int sk = (int)((walk + kMaxMomentItem - 1.0) / kMaxMomentItem);
    sk = std::max(sk, s.splitk_min);
    return std::max(1, std::min(sk, s.splitk_max));
}

// Every item of every field, in the queue order of order_items on
// `workers` blocks (moment items with the K splits of fused_splitk).
inline std::vector<FusedItem> fused_items(const std::vector<FieldShape> &shapes, int workers) {
    std::vector<FusedItem> all;
    std::vector<OrderItem> ord;
    for (int f = 0; f < (int)shapes.size(); ++f) {
        const FieldShape &s = shapes[f];
        const int sk = fused_splitk(s);
        auto add = [&](int st, int a, int b, int c) {
            // an expansion item costs its blocks' cost each
            ord.push_back({f, st, (int)all.size(), fused_cost(s, sk, st, a, b) * (st == 3 ? c : 1)});
            all.push_back({f, st, a, b, c});
        };
        for (int u = 0; u < s.split_units; u += kSplitUnitsPerItem)
            add(0, u, std::min(kSplitUnitsPerItem, s.split_units - u), 0);
        for (int z = 0; z < sk; ++z)
            for (int m = 0; m < s.rows1; ++m)
                for (int c = 0; c < s.units_e + s.units_o; ++c) add(1, c, m, z);
        for (int x = 0; x < s.scan_blocks; ++x) add(2, x, 0, 0);
        for (int a = 0; a < s.cols2; a += kExpansionUnitsPerItem)
            for (int m = 0; m < s.rows2; ++m) add(3, m, a, std::min(kExpansionUnitsPerItem, s.cols2 - a));
    }
    for (int i = 0; i < (int)ord.size(); ++i) ord[i].idx = i;
    const std::vector<int> q = order_items(ord, (int)shapes.size(), kFusedStages, workers);
    std::vector<FusedItem> out;
    out.reserve(q.size());
    for (int i : q) out.push_back(all[i]);
    return out;
}

}  // namespace mpg
