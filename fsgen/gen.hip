// Device side of the seeded synthetic-input generator.  Same integer recipe
// as the numpy implementation in __init__.py (SplitMix64 output function,
// Steele, Lea & Flood, OOPSLA 2014), so both produce identical bytes.
// Test and benchmark infrastructure: no part of the sort lives here.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kMix1 = 0xBF58476D1CE4E5B9ull;
constexpr uint64_t kMix2 = 0x94D049BB133111EBull;
constexpr uint64_t kHotThreshold = (9ull << 32) / 10ull;

__device__ __forceinline__ uint64_t rand64(uint64_t seed, uint64_t stream, uint64_t i) {
    uint64_t z = (seed ^ (stream * kGolden)) + (i + 1) * kGolden;
    z = (z ^ (z >> 30)) * kMix1;
    z = (z ^ (z >> 27)) * kMix2;
    return z ^ (z >> 31);
}

// number of thresholds <= x in the sorted 65535-entry table
__device__ __forceinline__ uint64_t count_le(const uint64_t* thr, uint64_t x) {
    uint32_t lo = 0, hi = 65535;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (thr[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename K>
__global__ void gen_keys(K* out, uint64_t n, int key_bits, int dist, uint64_t seed,
                         const uint64_t* table) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const int drop = 64 - key_bits;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t k;
        switch (dist) {
        case 0: k = rand64(seed, 0, i) >> drop; break;                      // uniform
        case 1: case 2: k = count_le(table, rand64(seed, 0, i)); break;     // gaussian, zipf
        case 3: k = rand64(seed, 1, 0) >> drop; break;                      // equal
        case 4: k = (i << 16) / n; break;                                   // presorted
        case 5: k = 65535ull - (i << 16) / n; break;                        // reverse
        case 6: k = rand64(seed, 0, i) >> 44; break;                        // small20
        default: {                                                          // hot90
            uint64_t x = rand64(seed, 0, i) >> drop;
            uint64_t y = rand64(seed, 3, i);
            k = ((y >> 32) < kHotThreshold) ? table[(y >> 8) & 255] : x;
        }
        }
        out[i] = (K)k;
    }
}

template <typename V>
__global__ void gen_index(V* out, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (V)i;
}

unsigned grid_for(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    return (unsigned)(g > 65536 ? 65536 : (g ? g : 1));
}

}  // namespace

extern "C" int fsgen_keys(void* out, uint64_t n, int key_bits, int dist, uint64_t seed,
                          const uint64_t* table, void* stream) {
    if (n == 0) return 0;
    if (!out) return 1;
    if ((dist == 1 || dist == 2 || dist == 7) && !table) return 1;
    if (dist < 0 || dist > 7) return 1;
    hipStream_t s = (hipStream_t)stream;
    switch (key_bits) {
    case 16: gen_keys<uint16_t><<<grid_for(n), 256, 0, s>>>((uint16_t*)out, n, 16, dist, seed, table); break;
    case 32: gen_keys<uint32_t><<<grid_for(n), 256, 0, s>>>((uint32_t*)out, n, 32, dist, seed, table); break;
    case 64: gen_keys<uint64_t><<<grid_for(n), 256, 0, s>>>((uint64_t*)out, n, 64, dist, seed, table); break;
    default: return 1;
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int fsgen_index(void* out, uint64_t n, int val_bytes, uint64_t reserved, void* stream) {
    (void)reserved;
    if (n == 0) return 0;
    if (!out) return 1;
    hipStream_t s = (hipStream_t)stream;
    if (val_bytes == 4) gen_index<uint32_t><<<grid_for(n), 256, 0, s>>>((uint32_t*)out, n);
    else if (val_bytes == 8) gen_index<uint64_t><<<grid_for(n), 256, 0, s>>>((uint64_t*)out, n);
    else return 1;
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
