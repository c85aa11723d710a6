// Work items of the X-stage kernels: which tiles of which channels each
// workgroup computes, wave by wave.  Built once per plan on the host and
// uploaded as a table; the kernels read their item by index.
#include "xcorr_host.h"


namespace xcorr {

int item_blocks(const WorkItem& it)
{
    int n = 0;
    for (int w = 0; w < kMaxWaves; ++w) n += __builtin_popcount(kind_mask(it.kind[w]));
    return n;
}

namespace {

WorkItem blank_item()
{
    WorkItem it;
    for (int k = 0; k < kSlots; ++k) { it.rb[k] = -1; it.ch[k] = 0; }
    for (int w = 0; w < kMaxWaves; ++w) { it.wi[w] = 0; it.wj[w] = 0; it.kind[w] = KIND_NONE; }
    it.pad[0] = it.pad[1] = it.pad[2] = 0;
    return it;
}

// Lower-triangle work items for W row blocks of 64 inputs, four waves per
// workgroup (fp16 and fp32 kernels).  Off-diagonal pairs of row-block pairs
// become four FULL tiles; a diagonal pair becomes two DIAG tiles plus the
// off-diagonal tile between them split in two halves, so that no wave of the
// workgroup carries more than 10 of 16 blocks.
void plan_items4(int W, std::vector<WorkItem>& items, int& ch_group)
{
    constexpr int kWaves = 4;
    items.clear();
    auto blank = blank_item;
    if (W == 1) {
        // one row block per channel: four channels per workgroup, one DIAG tile each
        ch_group = kWaves;
        WorkItem it = blank();
        for (int w = 0; w < kWaves; ++w) {
            it.rb[w] = 0;
            it.ch[w] = (int8_t)w;
            it.wi[w] = it.wj[w] = (int8_t)w;
            it.kind[w] = KIND_DIAG;
        }
        items.push_back(it);
        return;
    }
    ch_group = 1;
    const int SB = (W + 1) / 2;
    for (int R = 0; R < SB; ++R) {
        int rr[2], nr = 0;
        for (int k = 0; k < 2; ++k) if (2 * R + k < W) rr[nr++] = 2 * R + k;
        for (int S = 0; S <= R; ++S) {
            WorkItem it = blank();
            if (S < R) {
                int ss[2], ns = 0;
                for (int k = 0; k < 2; ++k) if (2 * S + k < W) ss[ns++] = 2 * S + k;
                int slot = 0;
                for (int k = 0; k < nr; ++k) it.rb[slot++] = (int16_t)rr[k];
                for (int k = 0; k < ns; ++k) it.rb[slot++] = (int16_t)ss[k];
                int w = 0;
                for (int a = 0; a < nr; ++a)
                    for (int b = 0; b < ns; ++b) {
                        it.wi[w] = (int8_t)a;
                        it.wj[w] = (int8_t)(nr + b);
                        it.kind[w] = KIND_FULL;
                        ++w;
                    }
            } else if (nr == 2) {
                it.rb[0] = (int16_t)rr[0];
                it.rb[1] = (int16_t)rr[1];
                it.wi[0] = 1; it.wj[0] = 0; it.kind[0] = KIND_HALF0;
                it.wi[1] = 1; it.wj[1] = 0; it.kind[1] = KIND_HALF1;
                it.wi[2] = 0; it.wj[2] = 0; it.kind[2] = KIND_DIAG;
                it.wi[3] = 1; it.wj[3] = 1; it.kind[3] = KIND_DIAG;
            } else {
                it.rb[0] = (int16_t)rr[0];
                it.wi[0] = 0; it.wj[0] = 0; it.kind[0] = KIND_DIAG;
            }
            items.push_back(it);
        }
    }
}

// Eight waves per workgroup (int8 kernel), one row block per channel: four
// channels per workgroup, each diagonal tile in two balanced DIAG_A / DIAG_B
// waves of 5 blocks.
void plan_items8_single(std::vector<WorkItem>& items, int& ch_group)
{
    items.clear();
    ch_group = 4;
    WorkItem it = blank_item();
    for (int s = 0; s < kSlots; ++s) {
        it.rb[s] = 0;
        it.ch[s] = (int8_t)s;
        for (int h = 0; h < 2; ++h) {
            it.wi[2 * s + h] = it.wj[2 * s + h] = (int8_t)s;
            it.kind[2 * s + h] = h ? KIND_DIAG_B : KIND_DIAG_A;
        }
    }
    items.push_back(it);
}

void plan_items8_paired(int W, std::vector<WorkItem>& items, int& ch_group)
{
    items.clear();
    // Two channels per group.  An off-diagonal pair of row-block pairs is
    // one item per channel.  The diagonal pairs of both channels share one
    // item: the full tile of each channel as two HALF waves (waves 0-3) and
    // each diagonal tile as one DIAG wave of 10 blocks (waves 4-7), so that
    // the item keeps every SIMD at 18 blocks instead of 9.  A step of an
    // item costs about the same whatever its MFMA count (its copies,
    // barrier and fragment reads do not shrink with it): a diagonal item of
    // one channel, 9 blocks per SIMD, took as long as an off-diagonal one.
    // Items run in list order on the workgroups of an XCD, so the list is
    // channel-major: the off-diagonal items of the first channel, the
    // shared diagonal items, then the off-diagonal items of the second
    // channel; the workgroups running at one time then mostly read one
    // channel.
    ch_group = 2;
    const int SB = (W + 1) / 2;
    auto super_rows = [&](int R, int* r) {
        int n = 0;
        for (int k = 0; k < 2; ++k) if (2 * R + k < W) r[n++] = 2 * R + k;
        return n;
    };
    auto off_items = [&](int c) {
        for (int R = 0; R < SB; ++R) {
            int rr[2], ss[2];
            const int nr = super_rows(R, rr);
            for (int S = 0; S < R; ++S) {
                const int ns = super_rows(S, ss);
                WorkItem it = blank_item();
                int slot = 0;
                for (int k = 0; k < nr; ++k) { it.ch[slot] = (int8_t)c; it.rb[slot++] = (int16_t)rr[k]; }
                for (int k = 0; k < ns; ++k) { it.ch[slot] = (int8_t)c; it.rb[slot++] = (int16_t)ss[k]; }
                int w = 0;
                for (int a = 0; a < nr; ++a)
                    for (int b = 0; b < ns; ++b)
                        for (int h = 0; h < 2; ++h) {
                            it.wi[w] = (int8_t)a;
                            it.wj[w] = (int8_t)(nr + b);
                            it.kind[w++] = h ? KIND_HALF1 : KIND_HALF0;
                        }
                items.push_back(it);
            }
        }
    };
    off_items(0);
    for (int R = 0; R < SB; ++R) {
        int rr[2];
        const int nr = super_rows(R, rr);
        WorkItem it = blank_item();
        if (nr == 2) {
            for (int c = 0; c < 2; ++c)
                for (int k = 0; k < 2; ++k) {
                    it.rb[2 * c + k] = (int16_t)rr[k];
                    it.ch[2 * c + k] = (int8_t)c;
                }
            for (int c = 0; c < 2; ++c)
                for (int h = 0; h < 2; ++h) {
                    it.wi[2 * c + h] = (int8_t)(2 * c + 1);
                    it.wj[2 * c + h] = (int8_t)(2 * c);
                    it.kind[2 * c + h] = h ? KIND_HALF1 : KIND_HALF0;
                }
            for (int s = 0; s < 4; ++s) {
                it.wi[4 + s] = it.wj[4 + s] = (int8_t)s;
                it.kind[4 + s] = KIND_DIAG;
            }
        } else {
            for (int c = 0; c < 2; ++c) {
                it.rb[c] = (int16_t)rr[0];
                it.ch[c] = (int8_t)c;
                for (int h = 0; h < 2; ++h) {
                    it.wi[2 * c + h] = it.wj[2 * c + h] = (int8_t)c;
                    it.kind[2 * c + h] = h ? KIND_DIAG_B : KIND_DIAG_A;
                }
            }
        }
        items.push_back(it);
    }
    off_items(1);
}

}  // namespace

// Work items of a plan, used by every launch.  int8 plans pair the
// diagonal items of two channels (more than one row block) or put four
// channels in one item (one row block).  Adding launches take the same
// table: they add into an int32 accumulator.  (When they read and wrote
// the int64 accumulator the paired items made them 6 % slower at the LWA
// size, and a second, single-channel table served them.)  With a static
// schedule the paired list also made the 2048-input 8-bit window 6 %
// slower, from L2 misses; with the per-XCD queue it makes it 1 % faster.
void plan_items(int path, int W, std::vector<WorkItem>& items, int& ch_group)
{
    if (path != XCORR_PATH_I8_MFMA) plan_items4(W, items, ch_group);
    else if (W == 1) plan_items8_single(items, ch_group);
    else plan_items8_paired(W, items, ch_group);
}

}  // namespace xcorr
