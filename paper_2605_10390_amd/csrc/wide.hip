// Kernels of the multi-word key sort (fs_sort_keys_wide / fs_sort_pairs_wide).
//
// A key of W 64-bit words (word 0 least significant) is sorted
// least-significant word first, each round a stable sort of one word paired
// with the current permutation (the digit order of Section II applied to
// 64-bit "digits", each itself sorted by the 8-bit-digit passes).  These
// kernels make the permutation, gather one word of every key through it
// (mapped into the requested order), and move whole keys and payloads
// through the final permutation.
#include "fs_device.hpp"
#include "fs_internal.hpp"

namespace fs {

namespace {

uint32_t grid_for(uint64_t n) {
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g < 16384 ? (g ? g : 1) : 16384);
}

template <typename P>
__global__ void k_iota(P* __restrict__ perm, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) perm[i] = (P)i;
}

// word w of key perm[i] (of key i when perm is null), mapped by the order
// masks of that word: the mask is neg when the key's top word has its top
// bit set, else pos
template <typename P>
__global__ void k_gather_word(const uint64_t* __restrict__ keys, uint32_t words, uint32_t w,
                              const P* __restrict__ perm, uint64_t* __restrict__ out, uint64_t n,
                              uint64_t pos, uint64_t neg) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const bool by_sign = pos != neg;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = perm ? (uint64_t)perm[i] : i;
        const uint64_t* key = keys + k * words;
        const uint64_t x = key[w];
        uint64_t m = pos;
        if (by_sign) m = (key[words - 1] >> 63) ? neg : pos;
        out[i] = x ^ m;
    }
}

// whole keys (and payloads) through the permutation
template <typename P>
__global__ void k_gather_keys(const uint64_t* __restrict__ keys_in, uint64_t* __restrict__ keys_out,
                              uint32_t words, const P* __restrict__ perm, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t total = n * words;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += stride) {
        const uint64_t i = j / words, w = j - i * words;
        keys_out[j] = keys_in[(uint64_t)perm[i] * words + w];
    }
}

template <typename P, typename V>
__global__ void k_gather_vals(const V* __restrict__ vals_in, V* __restrict__ vals_out, const P* __restrict__ perm,
                              uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        vals_out[i] = vals_in[perm[i]];
}

}  // namespace

hipError_t launch_iota(void* perm, int perm_bytes, uint64_t n, hipStream_t s) {
    if (perm_bytes == 4) k_iota<uint32_t><<<grid_for(n), 256, 0, s>>>(static_cast<uint32_t*>(perm), n);
    else k_iota<uint64_t><<<grid_for(n), 256, 0, s>>>(static_cast<uint64_t*>(perm), n);
    return hipGetLastError();
}

hipError_t launch_gather_word(const void* keys, uint32_t words, uint32_t w, const void* perm, int perm_bytes,
                              uint64_t* out, uint64_t n, uint64_t pos, uint64_t neg, hipStream_t s) {
    const uint64_t* k = static_cast<const uint64_t*>(keys);
    if (perm_bytes == 4)
        k_gather_word<uint32_t><<<grid_for(n), 256, 0, s>>>(k, words, w, static_cast<const uint32_t*>(perm), out,
                                                            n, pos, neg);
    else
        k_gather_word<uint64_t><<<grid_for(n), 256, 0, s>>>(k, words, w, static_cast<const uint64_t*>(perm), out,
                                                            n, pos, neg);
    return hipGetLastError();
}

hipError_t launch_gather_keys(const void* keys_in, void* keys_out, uint32_t words, const void* perm, int perm_bytes,
                              uint64_t n, hipStream_t s) {
    const uint64_t* ki = static_cast<const uint64_t*>(keys_in);
    uint64_t* ko = static_cast<uint64_t*>(keys_out);
    const uint32_t g = grid_for(n * words);
    if (perm_bytes == 4) k_gather_keys<uint32_t><<<g, 256, 0, s>>>(ki, ko, words, static_cast<const uint32_t*>(perm), n);
    else k_gather_keys<uint64_t><<<g, 256, 0, s>>>(ki, ko, words, static_cast<const uint64_t*>(perm), n);
    return hipGetLastError();
}

hipError_t launch_gather_vals(const void* vals_in, void* vals_out, int val_bytes, const void* perm, int perm_bytes,
                              uint64_t n, hipStream_t s) {
    const uint32_t g = grid_for(n);
    if (perm_bytes == 4) {
        const uint32_t* p = static_cast<const uint32_t*>(perm);
        if (val_bytes == 4)
            k_gather_vals<uint32_t, uint32_t><<<g, 256, 0, s>>>(static_cast<const uint32_t*>(vals_in),
                                                                static_cast<uint32_t*>(vals_out), p, n);
        else
            k_gather_vals<uint32_t, uint64_t><<<g, 256, 0, s>>>(static_cast<const uint64_t*>(vals_in),
                                                                static_cast<uint64_t*>(vals_out), p, n);
    } else {
        const uint64_t* p = static_cast<const uint64_t*>(perm);
        if (val_bytes == 4)
            k_gather_vals<uint64_t, uint32_t><<<g, 256, 0, s>>>(static_cast<const uint32_t*>(vals_in),
                                                                static_cast<uint32_t*>(vals_out), p, n);
        else
            k_gather_vals<uint64_t, uint64_t><<<g, 256, 0, s>>>(static_cast<const uint64_t*>(vals_in),
                                                                static_cast<uint64_t*>(vals_out), p, n);
    }
    return hipGetLastError();
}

}  // namespace fs
