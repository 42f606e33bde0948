// Host check of the run-time radix schedules (lf2_gen.hpp): every length
// 2^a 3^b 5^c up to the longest run-time line gets at least one schedule,
// each schedule uses only the butterflies the kernels have (2, 3, 4, 5, 8,
// 16) and multiplies out to the length, no schedule appears twice, and
// lengths with another prime factor get none.  Prints "ok <count>" or the
// first failure.
#include <stdio.h>

#include "../../paper_1508_05610_amd/csrc/lf2_gen.hpp"

using namespace lf2;

int main()
{
    int lengths = 0;
    for (int L = 1; L <= kGenMaxLen; ++L) {
        const std::vector<GSched> c = sched_candidates(L);
        int m = L;
        for (int p : {2, 3, 5})
            while (m % p == 0) m /= p;
        const bool f235 = m == 1;
        if (!f235) {
            if (!c.empty()) {
                printf("FAIL %d has schedules\n", L);
                return 1;
            }
            continue;
        }
        if (c.empty()) {
            printf("FAIL %d has no schedule\n", L);
            return 1;
        }
        for (size_t i = 0; i < c.size(); ++i) {
            if (!sched_valid(c[i], L)) {
                printf("FAIL %d schedule %zu invalid\n", L, i);
                return 1;
            }
            for (size_t j = 0; j < i; ++j) {
                bool same = c[i].n == c[j].n;
                for (int k = 0; same && k < c[i].n; ++k) same = c[i].r[k] == c[j].r[k];
                if (same) {
                    printf("FAIL %d duplicate schedule\n", L);
                    return 1;
                }
            }
        }
        ++lengths;
    }
    // the default of 512 spreads its bits evenly: 8 8 8; of 720: 16 then 3 3 5
    const GSched a = sched_candidates(512)[0], b = sched_candidates(720)[0];
    if (!(a.n == 3 && a.r[0] == 8 && a.r[1] == 8 && a.r[2] == 8)) {
        printf("FAIL default of 512\n");
        return 1;
    }
    if (!(b.n == 4 && b.r[0] == 16 && b.r[1] == 3 && b.r[2] == 3 && b.r[3] == 5)) {
        printf("FAIL default of 720\n");
        return 1;
    }
    GSched bad{};
    bad.n = 2;
    bad.r[0] = 9;
    bad.r[1] = 5;
    if (sched_valid(bad, 45)) {
        printf("FAIL radix 9 accepted\n");
        return 1;
    }
    printf("ok %d\n", lengths);
    return 0;
}
