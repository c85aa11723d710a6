// Host check of the X-stage work-item planner (xcorr_items.cpp): for every
// path, row-block counts 1..24 and channel counts 1..5, every 16x16 block (i >= j) of the lower triangle of every channel is
// computed by exactly one wave, no wave computes a block above the diagonal
// or outside the channels, each channel's blocks come from tiles of that
// channel, and a wave of the eight-wave int8 kernel never owns more than 10
// blocks (its register budget).
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include "xcorr_host.h"

#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

using namespace xcorr;

static int check(const char* what, int W, int n_ch, const std::vector<WorkItem>& items, int cg, int cap)
{
    std::map<std::tuple<int, int, int>, int> seen;
    const int groups = (n_ch + cg - 1) / cg;
    for (int g = 0; g < groups; ++g)
        for (const WorkItem& it : items)
            for (int w = 0; w < kMaxWaves; ++w) {
                const uint32_t m = kind_mask(it.kind[w]);
                if (!m) continue;
                if (__builtin_popcount(m) > cap) {
                    std::printf("%s W=%d: wave with %d blocks\n", what, W, __builtin_popcount(m));
                    return 1;
                }
                const int si = it.wi[w], sj = it.wj[w];
                if (si < 0 || si >= kSlots || sj < 0 || sj >= kSlots || it.rb[si] < 0 || it.rb[sj] < 0) {
                    std::printf("%s W=%d: wave %d reads an empty slot\n", what, W, w);
                    return 1;
                }
                if (it.ch[si] != it.ch[sj]) {
                    std::printf("%s W=%d: wave %d mixes channels\n", what, W, w);
                    return 1;
                }
                const int c = g * cg + it.ch[si];
                if (c >= n_ch) continue;                   // past the last channel: never stored
                for (int bi = 0; bi < 4; ++bi)
                    for (int bj = 0; bj < 4; ++bj) {
                        if (!((m >> (4 * bi + bj)) & 1u)) continue;
                        const int I = 4 * it.rb[si] + bi, J = 4 * it.rb[sj] + bj;
                        if (J > I || I >= 4 * W) {
                            std::printf("%s W=%d: block (%d, %d) outside the triangle\n", what, W, I, J);
                            return 1;
                        }
                        ++seen[std::make_tuple(c, I, J)];
                    }
            }
    for (int c = 0; c < n_ch; ++c)
        for (int I = 0; I < 4 * W; ++I)
            for (int J = 0; J <= I; ++J) {
                auto f = seen.find(std::make_tuple(c, I, J));
                const int n = f == seen.end() ? 0 : f->second;
                if (n != 1) {
                    std::printf("%s W=%d channels=%d: block (%d, %d) of channel %d computed %d times\n", what, W,
                                n_ch, I, J, c, n);
                    return 1;
                }
            }
    return 0;
}

int main()
{
    const int paths[] = {XCORR_PATH_I8_MFMA, XCORR_PATH_F16_MFMA, XCORR_PATH_F32};
    for (int path : paths)
        for (int W = 1; W <= 24; ++W) {
            std::vector<WorkItem> items;
            int cg = 0;
            plan_items(path, W, items, cg);
            // eight-wave int8 items: at most 10 blocks a wave (two waves
            // share a SIMD's registers); four-wave items: whole tiles
            const int cap = path == XCORR_PATH_I8_MFMA ? 10 : 16;
            for (int n_ch = 1; n_ch <= 5; ++n_ch)
                if (check("items", W, n_ch, items, cg, cap)) return 1;
        }
    std::printf("ok\n");
    return 0;
}
