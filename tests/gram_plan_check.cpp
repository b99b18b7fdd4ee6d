// Host check of the work plans of the Gram (plan_gram, lower tiles) and of
// the Hilbert coupling (plan_rect, all tiles of an M x N product): for many
// shapes and CU counts, on the tile size the plan chose (128, or 64 for small
// products), every tile of the product appears once, either whole or as all of
// its pieces; piece units are distinct and in range; the summing entries name
// the split tiles; per-XCD tile counts differ by at most one; the split tiles
// are those of each XCD's last round only (fewer than its slots), and the
// split round takes no longer than leaving it whole.  Exit status 0 when all
// hold.  Pure host code: no device is touched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <set>
#include <vector>

#include "gn_internal.h"

int main() {
    int bad = 0, plans = 0, split = 0;
    struct Shape { long M, N; bool lower; };
    std::vector<Shape> shapes;
    for (long M : {300L, 700L, 1154L, 2100L, 3842L, 3969L, 4097L, 4223L, 4548L, 4850L, 5000L, 8514L, 9000L, 12000L,
                   12738L, 16385L, 20001L, 50308L})
        shapes.push_back({M, M, true});
    // Hilbert coupling shapes (collocation points x parameters), ragged edges
    for (Shape r : {Shape{8192, 8513, false}, Shape{1024, 8513, false}, Shape{16384, 1153, false},
                    Shape{6657, 1153, false}, Shape{1000, 8513, false}, Shape{4097, 4223, false}, Shape{300, 100, false},
                    Shape{65536, 65, false}, Shape{1024, 1153, false}, Shape{777, 321, false}})
        shapes.push_back(r);
    for (const Shape &sh : shapes) {
        const long M = sh.M;
        for (int cus : {256, 304, 240, 80, 8}) {
            std::vector<int4> t;
            int64_t nwork = 0;
            int nsplit = 0, pieces = 0, T = 0;
            const bool ok = sh.lower ? gn::plan_gram(M, cus, t, nwork, nsplit, pieces, T)
                                     : gn::plan_rect(M, sh.N, cus, t, nwork, nsplit, pieces, T);
            const int Tc = gn::plan_tile_size(M, sh.N, sh.lower);
            const long tiles_m = (M + Tc - 1) / Tc, tiles_n = sh.lower ? tiles_m : (sh.N + Tc - 1) / Tc;
            const long tiles = tiles_m;
            const long lower = sh.lower ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
            if (!ok) {
                if (lower >= 64 && cus % 8 == 0 && (sh.lower || sh.N > 64)) {
                    printf("M %ld N %ld cus %d: no plan\n", M, sh.N, cus);
                    ++bad;
                }
                continue;
            }
            if (T != Tc || (T != 128 && T != 64) || pieces < 1 || pieces > 4) {
                printf("M %ld: tile %d (expected %d), pieces %d\n", M, T, Tc, pieces);
                ++bad;
            }
            ++plans;
            split += nsplit > 0;
            const long slots = 2L * (cus / 8);
            std::map<std::pair<int, int>, std::set<int>> seen;
            std::vector<long> whole_x(8, 0), piece_x(8, 0);
            std::vector<int> unit_seen((size_t)nsplit * pieces, 0);
            for (long b = 0; b < nwork; ++b) {
                const int4 e = t[b];
                if (e.y < 0) continue;
                if (e.y >= tiles || e.z < 0 || e.z >= tiles_n || (sh.lower && e.z > e.y)) {
                    printf("M %ld: tile (%d, %d) outside the lower triangle\n", M, e.y, e.z);
                    ++bad;
                    continue;
                }
                std::set<int> &s = seen[{e.y, e.z}];
                if (e.x < 0) {
                    if (!s.empty()) ++bad;
                    s.insert(-1);
                    ++whole_x[b % 8];
                } else {
                    if (e.x >= nsplit * pieces || e.w < 0 || e.w >= pieces || e.x % pieces != e.w) {
                        printf("M %ld: bad unit %d piece %d\n", M, e.x, e.w);
                        ++bad;
                        continue;
                    }
                    ++unit_seen[e.x];
                    if (s.count(e.w) || s.count(-1)) ++bad;
                    s.insert(e.w);
                    ++piece_x[b % 8];
                }
            }
            if ((long)seen.size() != lower) {
                printf("M %ld cus %d: %zu tiles covered of %ld\n", M, cus, seen.size(), lower);
                ++bad;
            }
            for (auto &kv : seen)
                if (!kv.second.count(-1) && (int)kv.second.size() != pieces) ++bad;
            for (int u : unit_seen)
                if (u != 1) {
                    ++bad;
                    break;
                }
            if ((long)t.size() != nwork + nsplit) ++bad;
            for (int i = 0; i < nsplit; ++i) {
                const int4 f = t[nwork + i];
                auto it = seen.find({f.y, f.z});
                if (f.x != i * pieces || it == seen.end() || it->second.count(-1)) ++bad;
            }
            long lo = 1L << 40, hi = 0;
            for (int x = 0; x < 8; ++x) {
                const long tiles_x = whole_x[x] + piece_x[x] / std::max(pieces, 1);
                lo = std::min(lo, tiles_x);
                hi = std::max(hi, tiles_x);
                // the split tiles are the last round's: fewer than the slots, and the
                // split round (units of 1 / pieces of a tile) no longer than one whole round
                const long split_x = piece_x[x] / std::max(pieces, 1);
                if (split_x >= slots || (pieces > 1 && (piece_x[x] + slots - 1) / slots > pieces)) {
                    printf("M %ld cus %d: %ld split tiles (%ld pieces) on XCD %d, %ld slots\n", M, cus, split_x,
                           piece_x[x], x, slots);
                    ++bad;
                }
            }
            if (hi - lo > 1) {
                printf("M %ld cus %d: tiles per XCD from %ld to %ld\n", M, cus, lo, hi);
                ++bad;
            }
        }
    }
    printf("%d plans (%d with split tiles): %s\n", plans, split, bad ? "FAILED" : "all invariants hold");
    return bad != 0;
}
