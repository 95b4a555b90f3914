// Column ranges covered by the BFS level launches of a batched global
// relabel (host code only; no HIP types, so it also builds with a plain C++
// compiler).
//
// The volumes of a batch are packed in order, volume i owning the global
// columns [col_base(i), col_base(i) + cols(i)).  A level launch covers at
// most `max_ranges` column ranges.  Each search keeps two per-volume flag
// vectors: `live` (the volume's search has not ended) and `cover` (every
// level so far has covered the volume).  cover_ranges() chooses the volumes
// that the next levels cover:
//   - every live volume;
//   - of the other volumes still in `cover`, only those in the smallest
//     gaps between runs of live volumes, as many gaps as keep the covered
//     volumes within `max_ranges` runs of consecutive volumes.
// `cover` only shrinks: a level may cover a column only if every earlier
// level covered it, because the record buffers of a column that a level
// skipped fall behind.  A gap may be joined only if all of its volumes are
// still in `cover`.  Since every live volume lies in `cover` and `cover`
// forms at most `max_ranges` runs, joining the gaps inside the runs of
// `cover` always brings the count within the bound.
//
// Runs of covered volumes become ranges: range r starts at column lo[r] and
// takes the launch threads pre[r] <= t < pre[r + 1] (pre[0] = 0).  `lo`
// holds max_ranges entries and `pre` max_ranges + 1.  Returns the number of
// ranges, or -1 (lo, pre and cover untouched) if more than max_ranges would
// be needed, which the invariant above rules out when `cover` meets it.
#pragma once
#include <algorithm>
#include <utility>
#include <vector>

namespace smf {

template <class ColBase, class Cols>
int cover_ranges(int n, ColBase col_base, Cols cols, const std::vector<char> &live,
                 std::vector<char> &cover, int max_ranges, int *lo, int *pre)
{
    std::vector<std::pair<int, int>> runs;   // first and last volume of each run of live volumes
    for (int i = 0; i < n; ++i) {
        if (!live[i]) continue;
        if (!runs.empty() && runs.back().second == i - 1) runs.back().second = i;
        else runs.push_back({i, i});
    }
    // gaps between consecutive runs whose volumes are all still covered,
    // by their column count
    std::vector<std::pair<long long, size_t>> gaps;   // (columns, run before the gap)
    for (size_t k = 0; k + 1 < runs.size(); ++k) {
        bool ok = true;
        long long ncols = 0;
        for (int i = runs[k].second + 1; i < runs[k + 1].first; ++i) {
            ok = ok && cover[i];
            ncols += cols(i);
        }
        if (ok) gaps.push_back({ncols, k});
    }
    std::sort(gaps.begin(), gaps.end());
    std::vector<char> join(runs.size(), 0);   // run k continues into run k + 1
    size_t nruns = runs.size();
    for (const auto &gp : gaps) {
        if (nruns <= (size_t)max_ranges) break;
        join[gp.second] = 1;
        --nruns;
    }
    if (nruns > (size_t)max_ranges) return -1;
    std::vector<char> next((size_t)n, 0);
    int nr = 0;
    pre[0] = 0;
    for (size_t k = 0; k < runs.size();) {
        size_t e = k;
        while (join[e]) ++e;
        const int a = runs[k].first, b = runs[e].second;
        for (int i = a; i <= b; ++i) next[i] = 1;
        lo[nr] = col_base(a);
        pre[nr + 1] = pre[nr] + (col_base(b) + cols(b) - col_base(a));
        ++nr;
        k = e + 1;
    }
    cover.swap(next);
    return nr;
}

}  // namespace smf
