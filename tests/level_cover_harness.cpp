// Test harness of paper_2601_17026_amd/csrc/level_cover.h: the same
// cover_ranges() the solver uses, over plain arrays, for a CPU test.
#include <vector>

#include "../paper_2601_17026_amd/csrc/level_cover.h"

extern "C" int level_cover(int n, const int *col_base, const int *cols, const signed char *live,
                           signed char *cover, int max_ranges, int *lo, int *pre)
{
    std::vector<char> l(live, live + n), c(cover, cover + n);
    const int nr = smf::cover_ranges(
        n, [&](int i) { return col_base[i]; }, [&](int i) { return cols[i]; }, l, c, max_ranges, lo, pre);
    for (int i = 0; i < n; ++i) cover[i] = c[i];
    return nr;
}
