// batch_ranges.hpp -- a large batched launch as several launches over
// consecutive ranges of its execution list (host code).
//
// A persistent grid that walks a long tile list drifts apart: its
// workgroups end up far from each other in the arrays, and the memory side
// serves them less well than a grid that walks a short list in step.
// Splitting the list into ranges of about kBatchRangeBytes per operand, each
// its own launch with the knobs tuned for its size, restarts the grid in
// step at every range (measured 5-16 % faster on groups of 2 GiB per
// operand; a list under two ranges' worth of elements stays one launch,
// where the extra launch would cost more than the drift). Every tile still runs exactly once and writes its own outputs
// and partial, so the results do not depend on the split; the per-item
// combine of the dots runs once, after the last range.
#pragma once

#include <cstdint>

#include "batch.hpp"

namespace salt {

constexpr int64_t kBatchRangeBytes = (int64_t)128 << 20;

// Tiles per range for tiles of tile_elems elements of es bytes, ranges of
// range_bytes per operand (0: kBatchRangeBytes; negative: never split), or
// 0 when the list runs as one launch: its items hold total_elems elements,
// fewer than two ranges' worth (the decision counts elements, not tiles,
// since a list of many short items has many partly filled tiles).
inline int64_t batch_range_tiles(int64_t total_elems, int64_t tile_elems, int64_t es, int64_t range_bytes = 0) {
    if (range_bytes < 0) return 0;
    const int64_t bytes = range_bytes > 0 ? range_bytes : kBatchRangeBytes;
    const int64_t per = bytes / (tile_elems * es);
    return per > 0 && total_elems * es >= 2 * bytes ? per : 0;
}

// Launch L's list (its items holding total_elems elements) as ranges with
// launch(range) (returns a hipError_t as int); knobs(elems, range) sets
// unroll, nontemporal and blocks for a launch of `elems` elements (about
// that many for a range: its tiles times the tile size) and returns 0, or a
// status.
template <class Launch, class Knobs>
int launch_batch_ranges(const Launch &fn, const BatchLaunch &L, int64_t total_elems, int64_t tile_elems,
                        int64_t es, const Knobs &knobs, int64_t range_bytes = 0) {
    const int64_t per = batch_range_tiles(total_elems, tile_elems, es, range_bytes);
    if (per == 0 || L.total_tiles < 2 * per) {
        BatchLaunch one = L;
        one.combine = 1;
        const int st = knobs(total_elems, one);
        return st ? st : fn(one);
    }
    const int64_t parts = L.total_tiles / per;  // the last range takes the remainder
    for (int64_t q = 0; q < parts; ++q) {
        BatchLaunch r = L;
        r.tiles = L.tiles + q * per;
        r.total_tiles = q + 1 < parts ? per : L.total_tiles - q * per;
        r.combine = q + 1 == parts ? 1 : 0;
        int st = knobs(r.total_tiles * tile_elems, r);
        if (st == 0) st = fn(r);
        if (st) return st;
    }
    return 0;
}

}  // namespace salt
