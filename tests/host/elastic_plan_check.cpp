// Host-side check of the elastic address-range bookkeeping (elastic.hpp) against a
// brute-force model: random slot sizes and granules, random acquire / release order.
// After every step the committed granules must be exactly those some in-use slot's range
// touches, every run released must have been committed whole before, and the plan's
// committed count must match. Prints one line and exits non-zero on a violation.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "elastic.hpp"

int main() {
    std::mt19937_64 rng(12345);
    int bad = 0, cases = 0;
    for (int trial = 0; trial < 400; ++trial) {
        const size_t gran = size_t(1) << (rng() % 6 + 4);  // 16 .. 512 bytes
        const int nslot = 1 + rng() % 12;
        const size_t per = 1 + rng() % (4 * gran);         // bytes per slot, any alignment
        const size_t base = rng() % (2 * gran);            // ranges start anywhere
        sapdd::ElasticPlan plan(gran, base + nslot * per);
        std::map<size_t, size_t> live;                      // committed runs: first -> n
        std::set<int> used;
        for (int step = 0; step < 60; ++step) {
            const int s = rng() % nslot;
            std::vector<sapdd::GranRun> runs;
            if (used.count(s)) {
                plan.release(base + s * per, per, runs);
                used.erase(s);
                for (auto &r : runs) {
                    auto it = live.find(r.g);
                    if (it == live.end() || it->second != r.n) ++bad;  // not committed whole
                    else live.erase(it);
                }
            } else {
                plan.acquire(base + s * per, per, runs);
                used.insert(s);
                for (auto &r : runs) {
                    for (auto &kv : live)  // no overlap with a committed run
                        if (r.g < kv.first + kv.second && kv.first < r.g + r.n) ++bad;
                    live[r.g] = r.n;
                }
            }
            std::set<size_t> want, have;
            for (int u : used)
                for (size_t g = (base + u * per) / gran; g < (base + (u + 1) * per + gran - 1) / gran; ++g) want.insert(g);
            size_t total = 0;
            for (auto &kv : live) {
                for (size_t g = kv.first; g < kv.first + kv.second; ++g) have.insert(g);
                total += kv.second;
            }
            if (want != have || total != plan.committed()) ++bad;
            ++cases;
        }
    }
    std::printf("%d steps checked, %d violations\n", cases, bad);
    return bad ? 1 : 0;
}
