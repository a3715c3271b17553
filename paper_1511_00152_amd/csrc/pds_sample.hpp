// Exact-m sampling without replacement (Sec. I setup; App. B) into LDS
// bitmaps, shared by the sampling kernel and the batched compression kernel.
//
// Floyd's algorithm (Bentley & Floyd, CACM 1987): for t = p-m .. p-1 draw r
// uniform on {0..t}; keep r, or keep t when r is already kept.  Draws are
// Lemire's method on the sample's own Philox word stream (key (seed, 0),
// counter (block, sample, 0, 0)), so the subset of a sample depends on
// (seed, sample, p, m) only.  Bitmap word w of column col lives at
// bitmap[w * stride + col].
#pragma once

#include "pds_device.hpp"

namespace pds {

// Exclusive prefix sum over the 64 lanes of a wave, on data-parallel
// primitives (no LDS round trips): shifts by 1, 2, 4, 8 within each row of
// 16 lanes, then each row's total broadcast to the rows above it.  Lanes whose
// source lies outside the pattern add zero.  All 64 lanes must be active.
__device__ inline int wave_exclusive_scan(int v)
{
    int x = v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return x - v;
}

// Eight draws of Floyd's loop from one Philox block (stream words 8 wb ..
// 8 wb + 7), while t < p and no word has stopped the fast path.  Each draw is
// written without branches: the words of c and of t are read together, and
// both are written back (the same value twice when they are one word), so
// independent Philox arithmetic placed around it fills the LDS round trips.
// A word whose low product half is below the range (the only words Lemire's
// method can reject, probability below range / 2^32 per draw) sets stop_word
// and ends the fast path there.
__device__ inline void floyd_draw8(const u64x4& blkw, uint64_t wb, int p, int& t, int64_t& stop_word,
                                   uint32_t* bitmap, int stride, int col)
{
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w[2 * q] = (uint32_t)blkw.w[q];
        w[2 * q + 1] = (uint32_t)(blkw.w[q] >> 32);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool act = t < p && stop_word < 0;
        const uint32_t range = (uint32_t)(t + 1);
        const uint64_t prod = (uint64_t)w[q] * range;
        const bool st = act && (uint32_t)prod < range;
        stop_word = st ? (int64_t)(wb * 8 + q) : stop_word;
        const bool go = act && !st;
        const uint32_t c = go ? (uint32_t)(prod >> 32) : 0u;
        const uint32_t tt = go ? (uint32_t)t : 0u;
        uint32_t* wc = &bitmap[(c >> 5) * stride + col];
        uint32_t* wt = &bitmap[(tt >> 5) * stride + col];
        const uint32_t bc = go ? 1u << (c & 31) : 0u;
        const uint32_t bt = 1u << (tt & 31);
        const uint32_t oc = *wc, ot = *wt;
        const bool hit = (oc & bc) != 0u;  // c already kept: keep t instead
        const bool same = wc == wt;
        const uint32_t nc = oc | (hit ? (same ? bt : 0u) : bc);
        const uint32_t nt = same ? nc : (ot | (hit ? bt : 0u));
        *wc = nc;
        *wt = nt;
        t += go ? 1 : 0;
    }
}

// The exact sequential stream from stop_word on, for a lane whose fast path
// stopped (Lemire's rejection handled word by word).
__device__ inline void floyd_finish(uint64_t seed, uint64_t sample, int p, int t, int64_t stop_word,
                                    uint32_t* bitmap, int stride, int col)
{
    WordStream ws;
    ws.init(seed, sample);
    ws.seek((uint64_t)stop_word);
    for (; t < p; ++t) {
        const uint32_t c = uniform_below(ws, (uint32_t)(t + 1));
        uint32_t* wc = &bitmap[(c >> 5) * stride + col];
        const uint32_t bit = 1u << (c & 31);
        if (*wc & bit)
            bitmap[((uint32_t)t >> 5) * stride + col] |= 1u << (t & 31);
        else
            *wc |= bit;
    }
}

// Kept set of one sample into a zeroed bitmap column (one lane's work).  Draw
// t uses word t - (p - m) of the stream while no word has stopped the fast
// path; the Philox block after the current one is computed during its draws.
__device__ inline void floyd_bitmap(uint64_t seed, uint64_t sample, int p, int m, uint32_t* bitmap, int stride,
                                    int col)
{
    uint64_t blk = 0;
    u64x4 cur = philox_block(0, sample, 0, 0, seed, 0);
    int t = p - m;
    int64_t stop_word = -1;
    while (t < p && stop_word < 0) {
        const u64x4 nxt = philox_block(blk + 1, sample, 0, 0, seed, 0);
        floyd_draw8(cur, blk, p, t, stop_word, bitmap, stride, col);
        cur = nxt;
        ++blk;
    }
    if (stop_word >= 0) floyd_finish(seed, sample, p, t, stop_word, bitmap, stride, col);
}

// The same kept set with two lanes per sample: lane l < 32 (owner) draws and
// owns bitmap column col; lane l + 32 (helper, same sample and column) only
// evaluates the odd Philox blocks, which reach the owner through a cross-lane
// read, so each lane computes one block per sixteen draws.  Called by the
// whole wave (the loop runs while any owner still draws; the cross-lane read
// needs both halves active).
__device__ inline void floyd_bitmap_pair(uint64_t seed, uint64_t sample, int p, int m, uint32_t* bitmap, int stride,
                                         int col, bool owner)
{
    const uint64_t half = owner ? 0 : 1;
    u64x4 cur = philox_block(half, sample, 0, 0, seed, 0);
    int t = p - m;
    int64_t stop_word = -1;
    for (uint64_t pr = 0;; ++pr) {
        if (__ballot(owner && t < p && stop_word < 0) == 0ull) break;
        const u64x4 nxt = philox_block(2 * pr + 2 + half, sample, 0, 0, seed, 0);
        u64x4 odd;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)cur.w[q], 32, 64);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(cur.w[q] >> 32), 32, 64);
            odd.w[q] = ((uint64_t)hi << 32) | lo;
        }
        if (owner) {
            floyd_draw8(cur, 2 * pr, p, t, stop_word, bitmap, stride, col);
            floyd_draw8(odd, 2 * pr + 1, p, t, stop_word, bitmap, stride, col);
        }
        cur = nxt;
    }
    if (owner && stop_word >= 0) floyd_finish(seed, sample, p, t, stop_word, bitmap, stride, col);
}

// Ascending emission of bitmap column col by the whole wave: each lane takes
// a contiguous run of bitmap words, a wave prefix sum of their popcounts gives
// its first output position, and emit(pos, coord) is called for each kept
// coordinate (lanes write side by side).  Called by all 64 lanes.
template <class F>
__device__ inline void emit_sorted(const uint32_t* bitmap, int stride, int col, int words, int lane, F emit)
{
    const int wpl = (words + 63) / 64;  // bitmap words per lane
    const int w0 = lane * wpl;
    int cnt = 0;
    for (int q = 0; q < wpl; ++q)
        if (w0 + q < words) cnt += __popc(bitmap[(w0 + q) * stride + col]);
    int pos = wave_exclusive_scan(cnt);
    for (int q = 0; q < wpl; ++q) {
        if (w0 + q >= words) break;
        uint32_t bits = bitmap[(w0 + q) * stride + col];
        while (bits) {
            const int b = __builtin_ctz(bits);
            emit(pos++, (w0 + q) * 32 + b);
            bits &= bits - 1u;
        }
    }
}

}  // namespace pds
