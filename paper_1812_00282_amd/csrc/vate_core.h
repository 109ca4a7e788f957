// Shared host/device helpers of the VATE HIP library: hashing, exact division
// by the block size, block index and block ACT.  Used by the kernels and by
// the host-side entry points (vate_host_hash / vate_host_block), so the host
// tests exercise exactly the code the GPU runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vate.h"

namespace vate {

constexpr uint32_t kPhi = 0x9E3779B9u;   // odd multiplier separating VAT indices

// MurmurHash3 32-bit finalizer (Appleby), written from its published
// description; the mix of both hash functions.
__host__ __device__ __forceinline__ uint32_t mix(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__host__ __device__ __forceinline__ uint32_t umulhi32(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}

// Exact unsigned division of 32-bit n by an invariant d >= 1 with one
// multiply-high, two shifts and two adds: Granlund & Montgomery, "Division by
// invariant integers using multiplication" (PLDI 1994), Sec. 4, Fig. 4.1.
// With l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1:
//     t = mulhi(m, n);  q = (t + ((n - t) >> s1)) >> s2,
// s1 = min(l, 1), s2 = max(l - 1, 0).  A divisor >= 2^32 (only possible for
// the block size when c = 32 and k = 1) is encoded so that q = 0.
struct Div32 {
    uint32_t m, s1, s2;
};

inline Div32 make_div32(uint64_t d)
{
    Div32 r;
    if (d >= (1ull << 32)) {         // n / d = 0 for every 32-bit n
        r.m = 0; r.s1 = 1; r.s2 = 31;
        return r;
    }
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    unsigned __int128 num = ((unsigned __int128)1 << 32) * ((1ull << l) - d);
    r.m = (uint32_t)(num / d + 1);
    r.s1 = l < 1 ? l : 1;
    r.s2 = l > 1 ? l - 1 : 0;
    return r;
}

__host__ __device__ __forceinline__ uint32_t div32(uint32_t n, Div32 d)
{
    uint32_t t = umulhi32(d.m, n);
    return (t + ((n - t) >> d.s1)) >> d.s2;
}

// Everything a kernel needs to know about one sketch, passed by value.
struct Geo {
    uint64_t N;          // 2^c ATs
    uint64_t a;          // Eq. 9 block size a, or a' of Fig. 5
    uint64_t thresh;     // Fig. 5: first pid of the (a'+1)-sized blocks
    uint32_t c, shift;   // shift = 32 - c
    uint32_t k, twok, g;
    uint32_t seed_a, seed_b;
    uint32_t partition;  // 0: Eq. 9-10, 1: Fig. 5
    uint32_t dr;         // 0: asynchronous timestamps; 1: distance recorders (VDRE)
    uint32_t wb;         // counter width in bits
    uint32_t blog;       // 0: independent VATs; b > 0: locality-blocked H (blocks of 2^b VATs)
    uint32_t base1;      // Fig. 5: index of the first (a'+1)-sized block, 2k - b'
    uint32_t fast_blocks;// every block but the last holds >= one 16-byte chunk
    Div32 div_a;         // divide by a (Eq. 9) or a' (Fig. 5)
    Div32 div_a1;        // divide by a' + 1 (Fig. 5)
};

// BH(bip) in [0, g): multiply-high range reduction of the mixed bip.
__host__ __device__ __forceinline__ uint32_t bh(const Geo &G, uint32_t bip)
{
    return umulhi32(mix(bip ^ G.seed_b), G.g);
}

// mix(aip ^ seed_a): the per-host part of H, computed once per host.
__host__ __device__ __forceinline__ uint32_t host_key(const Geo &G, uint32_t aip)
{
    return mix(aip ^ G.seed_a);
}

// H(aip, i) = top c bits of mix(host_key ^ i * phi).
__host__ __device__ __forceinline__ uint32_t vat_pid(const Geo &G, uint32_t key, uint32_t i)
{
    if (G.blog == 0) {
        const uint32_t x = mix(key ^ (i * kPhi));
        return x >> G.shift;                     // shift = 32 - c <= 31
    }
    // blocked: slot i mod 2^b of the block floor(i / 2^b), placed at the top
    // c - b bits of the block number's mix, times 2^b
    const uint32_t bm = (1u << G.blog) - 1u;
    const uint32_t x = mix(key ^ ((i >> G.blog) * kPhi));
    return ((x >> G.shift) & ~bm) | (i & bm);
}

// Block index of an AT (Eq. 9-10 with the last block taking the remainder,
// or the low-deviation partition of Fig. 5).
__host__ __device__ __forceinline__ uint32_t block_of(const Geo &G, uint32_t pid)
{
    if (G.partition == 0) {
        uint32_t q = div32(pid, G.div_a);
        return q < G.twok - 1 ? q : G.twok - 1;
    }
    if ((uint64_t)pid < G.thresh)
        return div32(pid, G.div_a);
    return G.base1 + div32((uint32_t)(pid - G.thresh), G.div_a1);
}

// First AT of block i (i in [0, 2k]; block 2k is the end of the pool).
__host__ __device__ __forceinline__ uint64_t block_start(const Geo &G, uint32_t i)
{
    if (i >= G.twok)
        return G.N;
    if (G.partition == 0)
        return (uint64_t)i * G.a;
    if (i <= G.base1)
        return (uint64_t)i * G.a;
    return G.thresh + (uint64_t)(i - G.base1) * (G.a + 1);
}

// ACT of block i at the current slice: (BACT^0 + i) mod 2k (Eq. 8).
__host__ __device__ __forceinline__ uint32_t block_act(const Geo &G, uint32_t bact0, uint32_t bid)
{
    uint32_t act = bact0 + bid;
    return act >= G.twok ? act - G.twok : act;
}

// Distance of a non-inactive value (Eq. 5): (ACT + 2k - Value) mod 2k.
__host__ __device__ __forceinline__ uint32_t at_dist(const Geo &G, uint32_t act, uint32_t v)
{
    int d = (int)act - (int)v;
    return (uint32_t)(d < 0 ? d + (int)G.twok : d);
}

// Value of a counter that is inactive for every window: 2k for an AT (Sec. 3),
// k for a DR (a DR saturates at k, which already exceeds every k' - 1).
__host__ __device__ __forceinline__ uint32_t inactive_value(const Geo &G)
{
    return G.dr ? G.k : G.twok;
}

// Distance of a stored value that is not inactive: Eq. 5 for an AT (from its
// block's ACT); the value itself for a DR.
__host__ __device__ __forceinline__ uint32_t value_dist(const Geo &G, uint32_t bact0, uint32_t pid, uint32_t v)
{
    return G.dr ? v : at_dist(G, block_act(G, bact0, block_of(G, pid)), v);
}

// Validate parameters and fill the geometry; returns VATE_OK or an error code
// with a static message in *why.
int make_geo(const vate_params *p, Geo *G, const char **why);

}  // namespace vate
