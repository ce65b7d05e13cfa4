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
// ----------------------------------------------------------------------------
__device__ inline void finish_plan(const uint64_t* h, int digits, uint64_t n, uint64_t* hist,
                            uint64_t* base, uint32_t* plan, bool clobber = false) {
    __shared__ uint64_t wsum[4];
    __shared__ uint32_t trivial[8];
    const int b = threadIdx.x;
    for (int j = 0; j < digits; ++j) {
        uint64_t total;
        const uint64_t start = scan256_exclusive<uint64_t>(b < kRadix ? h[j] : 0, wsum, &total);
        if (b < kRadix) {
            hist[j * kRadix + b] = h[j];
            base[(uint64_t)j * 2 * kRadix + b] = start;  // buffer 0 of pass j
        }
        const int any = __syncthreads_or(b < kRadix && h[j] == n);
        if (b == 0) trivial[j] = any;
    }
    __syncthreads();
    if (b == 0) {
        int active_count = 0;
        for (int j = 0; j < digits; ++j) active_count += trivial[j] ? 0 : 1;
        int i = 0;
        uint32_t prev = kBufIn;
        for (int j = 0; j < 16; ++j) {
            const bool act = j < digits && !trivial[j];
            plan[4 * j] = act ? 1u : 0u;
            plan[4 * j + 1] = 0;
            plan[4 * j + 2] = 0;
            plan[4 * j + 3] = 0;
            if (act) {
                const int from_out = clobber ? i : active_count - 1 - i;
                const uint32_t dst = (from_out % 2 == 0) ? kBufOut : kBufTmp;
                plan[4 * j + 1] = prev;
                plan[4 * j + 2] = dst;
                prev = dst;
                ++i;
            }
        }
        plan[kPlanCopy] = (active_count == 0 || (clobber && active_count % 2 == 0)) ? 1u : 0u;
    }
}

}  // namespace fs
