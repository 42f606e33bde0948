// lf2_gen.hpp -- radix schedules chosen at run time, for line lengths
// 2^a 3^b 5^c that have no compiled kernel (and as alternatives for those
// that do).  A schedule is the list of radices of the Stockham stages, in
// order; their product is the line length.  Plain C++ (host planning and
// the kernels' argument block).
#pragma once
#include <stdint.h>

#include <vector>

namespace lf2 {

constexpr int kGenMaxStages = 15;  // 2^a 3^b 5^c <= 2^20 needs at most 14 stages of radix >= 2
constexpr int kGenMaxLen = 8192;   // longest line of the run-time kernels

struct GSched {
    int32_t n;                  // number of stages
    int32_t r[kGenMaxStages];   // radices, each one of 2, 3, 4, 5, 8, 16
};

inline bool gen_factorable(int64_t L)
{
    if (L < 1) return false;
    for (int p : {2, 3, 5})
        while (L % p == 0) L /= p;
    return L == 1;
}

inline int64_t sched_product(const GSched &s)
{
    int64_t p = 1;
    for (int i = 0; i < s.n; ++i) p *= s.r[i];
    return p;
}

inline bool sched_valid(const GSched &s, int64_t L)
{
    if (s.n < 0 || s.n > kGenMaxStages) return false;
    for (int i = 0; i < s.n; ++i)
        if (s.r[i] != 2 && s.r[i] != 3 && s.r[i] != 4 && s.r[i] != 5 && s.r[i] != 8 &&
            s.r[i] != 16)
            return false;
    return sched_product(s) == L;
}

// Candidate schedules of a length, the default first:
//   0: the power-of-two part in ceil(a/4) stages with the bits spread evenly
//      (the compiled kernels' order), then the factors 3, then the 5s;
//   1: the odd factors first, then the power-of-two stages;
//   2: the power-of-two part in radix-8 stages (a radix 2 or 4 for the
//      rest), then the odd factors;
//   3: radix-16 stages first while they fit, then the rest, odd factors last.
// Duplicates are dropped.
inline std::vector<GSched> sched_candidates(int64_t L)
{
    std::vector<GSched> out;
    if (!gen_factorable(L) || L > kGenMaxLen) return out;
    int a = 0, b = 0, c = 0;
    int64_t m = L;
    while (m % 2 == 0) m /= 2, ++a;
    while (m % 3 == 0) m /= 3, ++b;
    while (m % 5 == 0) m /= 5, ++c;
    auto pow2_even = [&](std::vector<int> &v) {
        const int ns = (a + 3) / 4;
        for (int s = 0; s < ns; ++s) v.push_back(1 << (a / ns + (s < a % ns ? 1 : 0)));
    };
    auto odd = [&](std::vector<int> &v) {
        for (int i = 0; i < b; ++i) v.push_back(3);
        for (int i = 0; i < c; ++i) v.push_back(5);
    };
    std::vector<std::vector<int>> lists(4);
    pow2_even(lists[0]);
    odd(lists[0]);
    odd(lists[1]);
    pow2_even(lists[1]);
    {
        int k = a;
        while (k >= 3) lists[2].push_back(8), k -= 3;
        if (k) lists[2].push_back(1 << k);
        odd(lists[2]);
    }
    {
        int k = a;
        while (k >= 4) lists[3].push_back(16), k -= 4;
        if (k) lists[3].push_back(1 << k);
        odd(lists[3]);
    }
    for (auto &v : lists) {
        if ((int)v.size() > kGenMaxStages) continue;
        GSched s{};
        s.n = (int)v.size();
        for (int i = 0; i < s.n; ++i) s.r[i] = v[i];
        bool dup = false;
        for (auto &o : out) {
            bool same = o.n == s.n;
            for (int i = 0; same && i < s.n; ++i) same = o.r[i] == s.r[i];
            dup = dup || same;
        }
        if (!dup && sched_valid(s, L)) out.push_back(s);
    }
    return out;
}

}  // namespace lf2
