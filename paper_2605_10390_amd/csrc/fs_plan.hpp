// Device-side pass planning shared by the histogram paths.
#pragma once
#include "fs_device.hpp"

namespace fs {

// ----------------------------------------------------------------------------
// Plan: per digit, the exclusive prefix of its 256 bins (where each bin's
// block starts in the pass output) and whether the digit is trivial (one
// bin holds every key, so its stable scatter is the identity and the pass is
// skipped).  Active passes ping-pong between the output and the temporary
// buffer so that the last one lands in the output.  With `clobber` the
// temporary buffer is the input itself, so the first pass must write the
// output: passes then alternate output, input, output, ... and an even
// number of them ends in the input, which plan[kPlanCopy] then asks to be
// copied to the output.  At least 256 threads (all of the block call it);
// thread b < 256 owns bin b and h[j] is its count of digit j.
//
// trie_bits > 0 asks for the sparse-trie plan when it saves passes: the
// paper's trie needs only L = ceil(log2 n) levels (Section III-B.1) and
// leaves the remaining bits of each key as trailing bits sorted per bin
// (Algorithm 5).  Here the window is the top W = ceil(trie_bits / 8)
// non-trivial digits; when fewer digits than that are active, or a window
// digit has a bin holding more than twice a uniform digit's share (skewed
// keys, whose runs of equal window bits would be long and send the fixup to
// its fallback), the plain LSD plan is used.  Slot j of the plain plan sorts digit j (slots of trivial
// digits stay off).
// ----------------------------------------------------------------------------
__device__ inline void plan_chain(uint32_t* plan, int first_slot, const int* digit, int count, uint32_t start,
                                  bool last_to_out, bool active) {
    // each slot reads where the previous one wrote; destinations alternate
    // so that the chain's last pass writes the output when last_to_out, and
    // never write the buffer being read
    uint32_t prev = start;
    for (int i = 0; i < count; ++i) {
        uint32_t dst;
        if (last_to_out) dst = ((count - 1 - i) % 2 == 0) ? kBufOut : kBufTmp;
        else dst = (prev == kBufOut) ? kBufTmp : kBufOut;
        const int s = first_slot + i;
        plan[4 * s] = active ? 1u : 0u;
        plan[4 * s + 1] = prev;
        plan[4 * s + 2] = dst;
        plan[4 * s + 3] = (uint32_t)digit[i];
        prev = dst;
    }
}

__device__ inline uint32_t chain_end(const uint32_t* plan, int first_slot, int count, uint32_t start) {
    return count ? plan[4 * (first_slot + count - 1) + 2] : start;
}

__device__ inline void finish_plan(const uint64_t* h, int digits, uint64_t n, uint64_t* hist,
                            uint64_t* base, uint32_t* plan, bool clobber = false, int trie_bits = 0) {
    __shared__ uint64_t wsum[4];
    __shared__ uint32_t trivial[8], heavy[8];
    const int b = threadIdx.x;
    for (int j = 0; j < digits; ++j) {
        uint64_t total;
        const uint64_t start = scan256_exclusive<uint64_t>(b < kRadix ? h[j] : 0, wsum, &total);
        if (b < kRadix) {
            hist[j * kRadix + b] = h[j];
            base[(uint64_t)j * 2 * kRadix + b] = start;  // buffer 0 of pass j
        }
        const int any = __syncthreads_or(b < kRadix && h[j] == n);
        // a bin with more than twice a uniform digit's share: skewed keys,
        // whose window runs would be long
        const int hv = __syncthreads_or(b < kRadix && h[j] > n / 128);
        if (b == 0) {
            trivial[j] = any;
            heavy[j] = hv;
        }
    }
    __syncthreads();
    if (b == 0) {
        for (int w = 0; w < kPlanWords; ++w) plan[w] = 0;
        int act[8], a = 0;
        for (int j = 0; j < digits; ++j)
            if (!trivial[j]) act[a++] = j;
        const int W = (trie_bits + 7) / 8;
        bool skewed = false;
        for (int i = a - W; i < a; ++i) skewed |= i >= 0 && heavy[act[i]];
        if (trie_bits > 0 && W >= 1 && a > W && !skewed) {
            // window passes: the top W active digits, lowest first.  Without
            // clobber the chain ends in the output; with it the temporary
            // buffer is the input, so the chain starts at the output (out,
            // in, out, ...) and ends wherever its parity puts it
            plan_chain(plan, 0, act + (a - W), W, kBufIn, !clobber, true);
            const uint32_t X = chain_end(plan, 0, W, kBufIn);
            plan[kPlanTrie] = 1;
            plan[kPlanTrieShift] = 8u * (uint32_t)act[a - W];
            plan[kPlanFixBuf] = X;
            plan[kPlanCopyTmp] = X == kBufTmp ? 1u : 0u;
            // the fallback: an LSD over every active digit from X, off
            // until the fixup finds a run it cannot sort
            plan_chain(plan, kPlanCondSlot, act, a, X, false, false);
            plan[kPlanCondCopyTmp] = chain_end(plan, kPlanCondSlot, a, X) == kBufTmp ? 1u : 0u;
            plan[kPlanRecount0] = act[a - W] != 0 ? 1u : 0u;
        } else {
            // plain LSD: slot j sorts digit j when it is active
            int i = 0;
            uint32_t prev = kBufIn;
            for (int j = 0; j < digits; ++j) {
                plan[4 * j + 3] = (uint32_t)j;
                if (trivial[j]) continue;
                const int from_out = clobber ? i : a - 1 - i;
                const uint32_t dst = (from_out % 2 == 0) ? kBufOut : kBufTmp;
                plan[4 * j] = 1;
                plan[4 * j + 1] = prev;
                plan[4 * j + 2] = dst;
                prev = dst;
                ++i;
            }
            plan[kPlanCopy] = (a == 0 || (clobber && a % 2 == 0)) ? 1u : 0u;
        }
    }
}

}  // namespace fs
