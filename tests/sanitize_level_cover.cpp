// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of
// paper_2601_17026_amd/csrc/level_cover.h (tests/test_sanitizers.py): whole
// searches of random batches in which volumes end at random polls, with the
// range arrays sized exactly max_ranges (+1 for the prefix sums), so that a
// write past them is reported.
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2601_17026_amd/csrc/level_cover.h"

int main()
{
    std::mt19937 gen(1234);
    int bad = 0;
    for (int it = 0; it < 2000; ++it) {
        const int n = 1 + (int)(gen() % 40), max_ranges = 1 + (int)(gen() % 16);
        std::vector<int> base(n), cols(n);
        int acc = 0;
        for (int i = 0; i < n; ++i) {
            base[i] = acc;
            cols[i] = 1 + (int)(gen() % 50);
            acc += cols[i];
        }
        std::vector<char> live(n), cover(n, 1);
        for (int i = 0; i < n; ++i) live[i] = gen() % 3 != 0;
        while (true) {
            int *lo = new int[max_ranges];
            int *pre = new int[max_ranges + 1];
            const int nr = smf::cover_ranges(
                n, [&](int i) { return base[i]; }, [&](int i) { return cols[i]; }, live, cover,
                max_ranges, lo, pre);
            if (nr > max_ranges) ++bad;
            delete[] lo;
            delete[] pre;
            bool any = false;
            for (int i = 0; i < n; ++i) {
                if (live[i] && gen() % 4 == 0) live[i] = 0;
                any = any || live[i];
            }
            if (!any) break;
        }
    }
    std::printf("sanitized level cover runs: %d bad\n", bad);
    return bad != 0;
}
