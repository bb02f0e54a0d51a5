// Drives the batched runtime's host-only launch schedule (csrc/schedule.cpp)
// over many plan shapes; built with the address and undefined-behaviour
// sanitizers by tests/test_runtime_schedule.py.  Prints "ok" and exits 0 if
// every case is well formed.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "schedule.hpp"

using psl::SchedOp;

static int fail(const char* what, size_t nb, int np, unsigned nr) {
    std::printf("FAIL %s (nb %zu np %d n_rep %u)\n", what, nb, np, nr);
    return 1;
}

int main() {
    std::mt19937 rng(20150306);
    const size_t nbs[] = {0, 1, 2, 3, 5, 7, 31, 200};
    const int nps[] = {1, 2, 3, 4, 8};
    const unsigned nrs[] = {0, 1, 2, 10};
    for (size_t nb : nbs)
        for (int np : nps)
            for (unsigned nr : nrs)
                for (int trial = 0; trial < 3; ++trial) {
                    std::vector<uint32_t> sizes(nb);
                    for (auto& x : sizes) x = trial == 0 ? 4194304u : 1u + rng() % 5000000u;
                    const std::vector<int32_t> pipe = psl::assign_pipelines(sizes.data(), nb, np);
                    if (pipe.size() != nb) return fail("assignment size", nb, np, nr);
                    std::vector<unsigned long long> load(np > 0 ? size_t(np) : 1, 0);
                    unsigned long long biggest = 0;
                    for (size_t i = 0; i < nb; ++i) {
                        if (pipe[i] < 0 || pipe[i] >= (np > 1 ? np : 1))
                            return fail("pipeline out of range", nb, np, nr);
                        load[size_t(pipe[i])] += sizes[i];
                        if (sizes[i] > biggest) biggest = sizes[i];
                    }
                    // greedy largest-first: loads differ by at most the largest batch
                    unsigned long long lo = ~0ull, hi = 0;
                    for (auto l : load) {
                        lo = l < lo ? l : lo;
                        hi = l > hi ? l : hi;
                    }
                    if (np > 1 && nb >= size_t(np) && hi - lo > biggest)
                        return fail("unbalanced", nb, np, nr);
                    // with at least as many batches as pipelines none is idle
                    if (np > 1 && nb >= size_t(np))
                        for (auto l : load)
                            if (l == 0) return fail("idle pipeline", nb, np, nr);
                    const std::vector<SchedOp> ops = psl::build_schedule(sizes.data(), nb, np, nr);
                    const std::string bad = psl::check_schedule(ops, nb, np, nr);
                    if (!bad.empty()) return fail(bad.c_str(), nb, np, nr);
                }
    // the checker rejects malformed schedules
    std::vector<uint32_t> s3 = {10, 20, 30};
    std::vector<SchedOp> ops = psl::build_schedule(s3.data(), 3, 2, 2);
    std::vector<SchedOp> a = ops;
    a.erase(a.begin() + 2);                 // drop a batch
    if (psl::check_schedule(a, 3, 2, 2).empty()) return fail("missing batch accepted", 3, 2, 2);
    std::vector<SchedOp> b = ops;
    b[1].pipe = 5;                          // pipeline out of range
    if (psl::check_schedule(b, 3, 2, 2).empty()) return fail("bad pipeline accepted", 3, 2, 2);
    std::vector<SchedOp> c = ops;
    std::swap(c[4], c[5]);                  // fold before join
    if (psl::check_schedule(c, 3, 2, 2).empty()) return fail("fold before join accepted", 3, 2, 2);
    std::vector<SchedOp> d = ops;
    d.pop_back();                           // replica not closed
    if (psl::check_schedule(d, 3, 2, 2).empty()) return fail("open replica accepted", 3, 2, 2);
    std::printf("ok\n");
    return 0;
}
