// Work split and launch order of the convolution: which items (output row x
// m1 chunk x 64-cell group x k3 range) one launch processes, and in which
// order the workgroups reach the chip's eight XCDs.
#include <algorithm>
#include <vector>

#include "bz_internal.h"

namespace bz {

// Largest useful chunk count: the shortest kept m1 range of any row.
int max_chunks(int N) { return half_a1_end(N / 2 + 1); }

// Default split (bz_autotune / bz_set_split override it per batch size):
// for a few cells (small_by_default) the small-batch form (KH = 0) with
// enough chunks to fill the chip; above, four m1 chunks, which measured best or
// within a few per cent of the best for every mesh and batch of 256 - 1667
// cells, and at N <= 16 as many as every row allows (N = 16, 256 cells: 231
// us per convolution with 5 chunks, 243 us with 4, for 3 us more in the
// inverse transform, which adds one more partial sum; within 1 % of 4 chunks
// at 512 and 1024 cells); two k3 ranges at N = 32,
// where a whole row's accumulators and v line hold the wavefronts to one per
// SIMD, and four at N = 48, the only count compiled there.
Split choose_split(const bz_op *op, int64_t cellpad, int64_t ncells) {
    for (const auto &t : op->tuned)
        if (t.first == cellpad) {
            if (t.second.second == 0 && ncells > kSmallMaxCells) break;  // not for this many cells
            return {t.second.first, t.second.second};
        }
    const int N = op->N;
    if (small_by_default(N, ncells)) return {small_default_chunks(N, ncells), 0};
    const int KH = N >= 48 ? 4 : (N >= 32 ? 2 : 1);
    return {N <= 16 ? max_chunks(N) : std::min(4, max_chunks(N)), KH};
}

// valid (k3, m3) pairs of one line whose output k3 lies in range h of KH
int range_pairs(int N, int KH, int h) {
    const int kb = h * (N / KH), ke = (h + 1) * (N / KH);
    int n = 0;
    for (int m = 0; m < N; ++m) n += std::max(0, std::min(khi(N, m), ke - 1) - std::max(klo(N, m), kb) + 1);
    return n;
}

// Convolution schedule.  Workgroups are handed to the 8 XCDs of the chip in
// round-robin order (workgroup b runs on XCD b mod 8), and each XCD has its
// own L2.  The items (row, chunk, group, k3 range) are sorted group-major and cut into 8
// contiguous parts of equal cost, so each XCD works on as few cell groups as
// possible and their f^ lines stay in its L2; inside a part the items run
// heaviest first (longest-processing-time order) so the dispatcher balances
// rows of unequal length.  Part x is laid out at workgroups 8i + x; shorter
// parts are padded with empty items (row = -1).
namespace {

struct Entry {
    int64_t cost;
    ConvItem it;
};

// the items of rows [row0, row1) of one op, group-major, with their cost
// (kept lines x pairs of a line in the item's k3 range, + one line of fixed
// cost), appended to `all`
void append_entries(std::vector<Entry> &all, int64_t &total, int N, int64_t cellpad, int S, int KH, int row0,
                    int row1, int op) {
    const int G = (int)(cellpad / kWave);
    for (int g = 0; g < G; ++g)
        for (int r = row0; r < row1; ++r) {
            const int c1 = mcount(N, r / N), c2 = mcount(N, r % N);
            const int h = half_a1_end(c1);
            const int per = (h + S - 1) / S;
            for (int s = 0; s < S; ++s) {
                int64_t lines = 1;
                for (int a1 = s * per; a1 < std::min(h, (s + 1) * per); ++a1) lines += half_a2_end(c1, c2, a1);
                for (int q = 0; q < KH; ++q) {
                    const int64_t cost = lines * range_pairs(N, KH, q);
                    all.push_back({cost, ConvItem{r, s, g, q, op}});
                    total += cost;
                }
            }
        }
}

// cut the list into kXcds contiguous parts of (nearly) equal cost, order
// each part heaviest first, and interleave: part x at workgroups 8i + x
std::vector<ConvItem> order_for_xcds(const std::vector<Entry> &all, int64_t total) {
    std::vector<std::vector<Entry>> part(kXcds);
    int64_t acc = 0;
    for (const Entry &e : all) {
        const int x = (int)std::min<int64_t>(kXcds - 1, (acc * kXcds) / std::max<int64_t>(total, 1));
        part[x].push_back(e);
        acc += e.cost;
    }
    size_t longest = 0;
    for (auto &p : part) {
        std::stable_sort(p.begin(), p.end(), [](const Entry &a, const Entry &b) { return a.cost > b.cost; });
        longest = std::max(longest, p.size());
    }
    std::vector<ConvItem> items(longest * kXcds, ConvItem{-1, 0, 0, 0, 0});
    for (int x = 0; x < kXcds; ++x)
        for (size_t i = 0; i < part[x].size(); ++i) items[i * kXcds + x] = part[x][i].it;
    return items;
}

}  // namespace

std::vector<ConvItem> make_items(int N, int64_t cellpad, int S, int KH, int row0, int row1) {
    std::vector<Entry> all;
    int64_t total = 0;
    append_entries(all, total, N, cellpad, S, KH, row0, row1, 0);
    return order_for_xcds(all, total);
}

// A mixed launch: each op's items (all rows, group-major) are cut into
// kXcds contiguous parts of equal cost, and XCD x takes part x of every op,
// so every XCD gets the same mix of meshes (the time per term differs
// between meshes, so equal-cost parts of different meshes would not finish
// together) and, per op, as few cell groups as possible.  Inside an XCD's
// share the heaviest items (the largest N) start first.
std::vector<ConvItem> make_mixed_items(const std::vector<MixPart> &parts) {
    std::vector<std::vector<Entry>> part(kXcds);
    for (size_t j = 0; j < parts.size(); ++j) {
        std::vector<Entry> all;
        int64_t total = 0;
        append_entries(all, total, parts[j].N, parts[j].cellpad, parts[j].S, parts[j].KH, 0,
                       parts[j].N * parts[j].N, (int)j);
        int64_t acc = 0;
        for (const Entry &e : all) {
            const int x = (int)std::min<int64_t>(kXcds - 1, (acc * kXcds) / std::max<int64_t>(total, 1));
            part[x].push_back(e);
            acc += e.cost;
        }
    }
    size_t longest = 0;
    for (auto &p : part) {
        std::stable_sort(p.begin(), p.end(), [](const Entry &a, const Entry &b) { return a.cost > b.cost; });
        longest = std::max(longest, p.size());
    }
    std::vector<ConvItem> items(longest * kXcds, ConvItem{-1, 0, 0, 0, 0});
    for (int x = 0; x < kXcds; ++x)
        for (size_t i = 0; i < part[x].size(); ++i) items[i * kXcds + x] = part[x][i].it;
    return items;
}

// Windows of a stored table: the slabs of max_elems weights, merged with
// their successors until each window has at least min_rows rows, so that a
// launch over one window still has enough items to fill the chip.
std::vector<int> window_bounds(const std::vector<int64_t> &rowoff, int64_t total, int64_t max_elems, int min_rows) {
    const std::vector<int> b = slab_bounds(rowoff, total, max_elems);
    if (b.empty()) return b;
    std::vector<int> w{0};
    for (size_t j = 1; j < b.size(); ++j)
        if (b[j] - w.back() >= min_rows || j + 1 == b.size()) w.push_back(b[j]);
    // a short last window joins the one before it
    if (w.size() > 2 && w[w.size() - 1] - w[w.size() - 2] < min_rows) w.erase(w.end() - 2);
    return w;
}

// A launch of at least this many items keeps every SIMD of the chip busy
// for several rounds (1024 SIMDs, 2 - 3 wavefronts each at N >= 24); the
// byte windows of N = 32 (154 - 334 rows, 15 000 - 20 000 items for 512
// cells) stay as they are.
constexpr int64_t kFillItems = 8192;

int fill_rows(int64_t cellpad, int S, int KH) {
    const int64_t per_row = std::max<int64_t>(1, (cellpad / kWave) * S * KH);
    return (int)((kFillItems + per_row - 1) / per_row);
}

// Slabs of an op whose weights are computed on the fly: consecutive rows,
// each slab as many as fit max_elems packed weights.
std::vector<int> slab_bounds(const std::vector<int64_t> &rowoff, int64_t total, int64_t max_elems) {
    const int rows = (int)rowoff.size();
    std::vector<int> b{0};
    for (int r = 0; r < rows; ++r) {
        const int64_t end = r + 1 < rows ? rowoff[r + 1] : total;
        if (end - rowoff[r] > max_elems) return {};
        if (end - rowoff[b.back()] > max_elems) b.push_back(r);
    }
    b.push_back(rows);
    return b;
}

}  // namespace bz
