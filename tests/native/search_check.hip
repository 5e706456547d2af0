// Host check of the joins' batched list search (in_sorted_many, every tail
// form and arity the kernels use) and of the single search (in_sorted)
// against a linear scan, on random ascending lists at every alignment of
// the list base, lists that end at the array's last element included (the
// vector tail reads up to CI_PAD elements past it).  Exit status 0 when
// every answer agrees.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "join_device.h"

using namespace gsi;

int main() {
    std::mt19937 rng(12345);
    long bad = 0, tests = 0;
    for (int trial = 0; trial < 3000; trial++) {
        std::vector<uint32_t> v;
        std::vector<std::pair<uint32_t, uint32_t>> lists;
        const int nl = 1 + (int)(rng() % 8);
        for (int l = 0; l < nl; l++) {
            const uint32_t len = (rng() % 2) ? rng() % 20 : rng() % 300;
            std::vector<uint32_t> pool(500);
            for (uint32_t i = 0; i < 500; i++) pool[i] = i;
            std::shuffle(pool.begin(), pool.end(), rng);
            std::vector<uint32_t> li(pool.begin(), pool.begin() + len);
            std::sort(li.begin(), li.end());
            lists.push_back({(uint32_t)v.size(), len});
            v.insert(v.end(), li.begin(), li.end());
        }
        if (v.empty()) v.push_back(0);
        const uint32_t total = (uint32_t)v.size();
        // 256-byte aligned, CI_PAD spare elements (junk) after the last list
        const size_t bytes = ((total + CI_PAD) * 4 + 255) / 256 * 256;
        uint32_t *mem = static_cast<uint32_t *>(aligned_alloc(256, bytes));
        for (uint32_t i = 0; i < total; i++) mem[i] = v[i];
        for (uint32_t i = 0; i < CI_PAD; i++) mem[total + i] = rng();
        const uint32_t shift = rng() % 4;  // a label's lists need not start 16-byte aligned
        for (auto &L : lists) {
            if (L.first < shift) continue;
            const uint32_t *base = mem + shift;
            uint32_t st[2] = {L.first - shift, L.first - shift}, len[2] = {L.second, L.second};
            for (uint32_t x = 0; x < 510; x += 1 + rng() % 3) {
                const uint32_t xs[2] = {x, x + 1};
                bool h[4][2];
                in_sorted_many<2, true, 4>(base, st, len, xs, h[0]);
                in_sorted_many<2, true, 8>(base, st, len, xs, h[1]);
                in_sorted_many<2, false, 8>(base, st, len, xs, h[2]);
                in_sorted_many<2, false, 4>(base, st, len, xs, h[3]);
                for (int u = 0; u < 2; u++) {
                    bool lin = false;
                    for (uint32_t t = 0; t < len[u]; t++) lin |= base[st[u] + t] == xs[u];
                    const bool one = in_sorted(base + st[u], len[u], xs[u]);
                    tests++;
                    bool ok = one == lin;
                    for (int f = 0; f < 4; f++) ok = ok && h[f][u] == lin;
                    if (!ok) bad++;
                }
            }
        }
        free(mem);
    }
    printf("searches %ld, disagreements %ld\n", tests, bad);
    return bad != 0;
}
