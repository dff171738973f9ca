// Randomised test of the pool's range allocator (paper_2609_07842_amd/csrc/arena.h) against
// a plain occupancy bitmap: first fit, coalescing of returned ranges, and no overlap.
// Built and run under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py; prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

static int fail(const char *what, long a, long b)
{
    std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
    return 1;
}

int main()
{
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const int64_t cap = 1 + (int64_t)(rng() % 4000);
        vbc::Arena A;
        A.init(cap);
        std::vector<char> used((size_t)cap, 0);
        std::vector<std::pair<int64_t, int64_t>> held;
        for (int op = 0; op < 400; ++op) {
            if (held.empty() || rng() % 3 != 0) {
                const int64_t n = 1 + (int64_t)(rng() % (cap / 4 + 1));
                // the model's first fit: lowest start of a run of n free indices
                int64_t want = -1, run = 0;
                for (int64_t i = 0; i < cap; ++i) {
                    run = used[(size_t)i] ? 0 : run + 1;
                    if (run == n) { want = i - n + 1; break; }
                }
                const int64_t got = A.take(n);
                if (got != want) return fail("first fit", (long)got, (long)want);
                if (got >= 0) {
                    for (int64_t i = got; i < got + n; ++i) used[(size_t)i] = 1;
                    held.emplace_back(got, n);
                }
            } else {
                const size_t k = (size_t)(rng() % held.size());
                const auto h = held[k];
                held.erase(held.begin() + (long)k);
                A.give(h.first, h.second);
                for (int64_t i = h.first; i < h.first + h.second; ++i) used[(size_t)i] = 0;
            }
            // the free map equals the model's maximal free runs, none touching another
            int64_t pos = 0, prev_end = -1;
            for (const auto &f : A.free) {
                if (f.first < pos || f.second <= 0 || f.first + f.second > cap) return fail("range", (long)f.first, (long)f.second);
                if (f.first == prev_end) return fail("not coalesced", (long)f.first, (long)prev_end);
                for (int64_t i = pos; i < f.first; ++i)
                    if (!used[(size_t)i]) return fail("free index missing", (long)i, (long)f.first);
                for (int64_t i = f.first; i < f.first + f.second; ++i)
                    if (used[(size_t)i]) return fail("used index listed free", (long)i, (long)f.first);
                pos = prev_end = f.first + f.second;
            }
            for (int64_t i = pos; i < cap; ++i)
                if (!used[(size_t)i]) return fail("free tail missing", (long)i, (long)cap);
        }
        for (const auto &h : held) A.give(h.first, h.second);
        if (A.free.size() != 1 || A.free.begin()->first != 0 || A.free.begin()->second != cap)
            return fail("all returned", (long)A.free.size(), (long)cap);
    }
    std::printf("ok\n");
    return 0;
}
