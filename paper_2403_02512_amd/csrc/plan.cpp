// Pass planner: groups consecutive gate applications (and, in the adjoint
// sweep, generator inner products) into passes over LDS tiles.
//
// A pass owns a set S of b index bits that always contains the lowest
// coalescing bits.  Each tile holds the 2^b amplitudes that agree on all bits
// outside S, so any gate whose targets lie in S, with controls anywhere, and
// any diagonal gate, can be applied inside the tile.  The planner scans the
// item list in order and pulls an item into the current pass when it commutes
// with every item it skips over (paper Sec. 2.1.1: updates on disjoint index
// sets are independent).  Two items commute when every index bit they share
// is acted on diagonally by both (controls and diagonal targets); this is the
// GPU analogue of the paper's intra-/inter-register split (Sec. 2.1.2): the
// bits in S are the "intra" ones of this pass.
#include <algorithm>

#include "qsv_internal.h"

namespace qsv {

static bool is_diag(const std::vector<cd>& m, int dim) {
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            if (r != c && m[(size_t)r * dim + c] != cd(0.0, 0.0)) return false;
    return true;
}

Item make_item(const Factor& f, bool dot, int fidx, int n) {
    Item it;
    it.dot = dot;
    it.f = fidx;
    uint64_t tb = 0, cb = 0;
    for (int i = 0; i < f.k; ++i) tb |= 1ull << (n - 1 - f.tw[i]);
    for (int j = 0; j < f.nc; ++j) cb |= 1ull << (n - 1 - f.cw[j]);
    const bool diag = is_diag(dot ? f.g : f.m, 1 << f.k);
    it.xbits = diag ? 0 : tb;
    it.zbits = cb | (diag ? tb : 0);
    it.zrot = f.zrot && !dot;
    return it;
}

std::vector<Pass> plan_passes(const std::vector<Item>& items, int n, const PlanOptions& opt) {
    std::vector<Pass> passes;
    if (items.empty()) return passes;
    const int b = std::min(opt.b, n);
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
    const uint64_t low = (1ull << std::min(opt.low, b)) - 1;
    std::vector<char> done(items.size(), 0);
    size_t first = 0, left = items.size();
    while (left) {
        while (done[first]) ++first;
        Pass p;
        p.S = n <= b ? all : low;
        if (!opt.fusion) {
            // one factor per pass: an inner product travels with its un-apply
            size_t j = first;
            p.items.push_back((int)j);
            done[j] = 1;
            --left;
            if (items[j].dot && j + 1 < items.size() && !items[j + 1].dot && items[j + 1].f == items[j].f) {
                p.items.push_back((int)(j + 1));
                done[j + 1] = 1;
                --left;
            }
            for (int i : p.items) p.S |= items[i].xbits;
        } else {
            uint64_t bx = 0, bz = 0;
            int scanned = 0;
            int64_t lds = 0;  // slot accumulators and phase tables of the pass
            for (size_t j = first; j < items.size() && scanned < opt.max_scan; ++j) {
                if (done[j]) continue;
                ++scanned;
                const Item& it = items[j];
                const int64_t cost = (it.dot ? opt.slot_bytes : 0) + (it.zrot ? opt.ztab_bytes : 0);
                bool ok = !(it.xbits & (bx | bz)) && !(it.zbits & bx) && lds + cost <= opt.lds_budget;
                if (ok && it.xbits) {
                    const uint64_t ns = p.S | it.xbits;
                    if (__builtin_popcountll(ns) <= b)
                        p.S = ns;
                    else if (p.items.empty() && !bx && !bz && __builtin_popcountll(it.xbits) <= b)
                        p.S = it.xbits;  // a wide first gate: its targets first, low bits as room allows
                    else
                        ok = false;
                }
                if (ok) {
                    p.items.push_back((int)j);
                    done[j] = 1;
                    --left;
                    lds += cost;
                } else {
                    bx |= it.xbits;
                    bz |= it.zbits;
                    if (bx == all) break;
                }
            }
        }
        int bp = b;
        if (p.items.empty()) {
            // the first pending item does not fit next to the coalescing bits:
            // give it a pass of its own whose bit set starts from its targets
            const Item& it = items[first];
            p.S = it.xbits;
            bp = std::max(b, __builtin_popcountll(it.xbits));
            p.items.push_back((int)first);
            done[first] = 1;
            --left;
        }
        // pad S with the lowest free bits up to the tile width: longer contiguous runs
        for (int bit = 0; __builtin_popcountll(p.S) < bp && bit < n; ++bit) p.S |= 1ull << bit;
        passes.push_back(std::move(p));
    }
    return passes;
}

}  // namespace qsv
