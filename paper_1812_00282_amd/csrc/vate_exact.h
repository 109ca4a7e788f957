// Exact-width counters: an AT of ceil(log2(2k+1)) bits (a DR of
// ceil(log2(k+1)) bits) packed back to back, as the paper sizes its pool
// (Sec. 3: 2k+1 values per AT; Sec. 5: 10-bit ATs at k = 300).  Counter p
// sits at bits [p w, (p+1) w) of the pool read as little-endian 32-bit words,
// so a group of 32 counters fills exactly w words and starts on a word.
// Included into vate.hip inside namespace vate; the width w = G.wb is a
// run-time value (template width 0 selects these paths).
//
// Streaming kernels (init, census, preservation, DR maintenance) give each
// thread whole groups: the group's w words are read in order through a
// 64-bit bit buffer and, where counters change, written back the same way.
// SetAT writes the w bits of one counter, which may straddle two words, with
// an atomic OR of its set bits then an atomic AND of its clear bits on each
// word: every writer of a counter within a slice writes the same value, so
// the counter ends at that value under any interleaving, and the bits of
// neighbouring counters are never touched.

__device__ __forceinline__ uint32_t low_mask(uint32_t w) { return w >= 32 ? ~0u : (1u << w) - 1u; }

// Value of counter pid from 32-bit words (global or LDS).
__device__ __forceinline__ uint32_t load_x(const uint32_t *__restrict__ words, uint64_t pid, uint32_t wb)
{
    const uint64_t o = pid * wb;
    const uint32_t *p = words + (o >> 5);
    const uint32_t sh = (uint32_t)o & 31u;
    uint32_t v = p[0] >> sh;
    if (sh + wb > 32) v |= p[1] << (32 - sh);
    return v & low_mask(wb);
}

__device__ __forceinline__ void set_x(uint32_t *__restrict__ words, uint64_t pid, uint32_t wb, uint32_t val)
{
    const uint64_t o = pid * wb;
    uint32_t *p = words + (o >> 5);
    const uint32_t sh = (uint32_t)o & 31u;
    const uint32_t n0 = min(wb, 32u - sh);             // bits in the first word
    const uint32_t m0 = low_mask(n0);
    atomicOr(p, (val & m0) << sh);
    atomicAnd(p, ~((~val & m0) << sh));
    if (n0 < wb) {
        const uint32_t m1 = low_mask(wb - n0), hi = val >> n0;
        atomicOr(p + 1, hi & m1);
        atomicAnd(p + 1, ~(~hi & m1));
    }
}

// The 32 counters of group gi (its wb words in order).
__device__ __forceinline__ void read_group(const uint32_t *__restrict__ src, uint32_t wb, uint32_t vals[32])
{
    uint64_t buf = 0;
    uint32_t have = 0;
    const uint32_t m = low_mask(wb);
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        if (have < wb) {
            buf |= (uint64_t)(*src++) << have;
            have += 32;
        }
        vals[e] = (uint32_t)buf & m;
        buf >>= wb;
        have -= wb;
    }
}

__device__ __forceinline__ void write_group(uint32_t *__restrict__ dst, uint32_t wb, const uint32_t vals[32])
{
    uint64_t buf = 0;
    uint32_t have = 0;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        buf |= (uint64_t)vals[e] << have;
        have += wb;
        if (have >= 32) {
            *dst++ = (uint32_t)buf;
            buf >>= 32;
            have -= 32;
        }
    }
}

// InitAT on every counter, clock and census reset.
__global__ void __launch_bounds__(256) k_init_x(Geo G, uint32_t *__restrict__ pool32, uint64_t ngroups,
                                                DevState *__restrict__ st)
{
    uint32_t vals[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) vals[e] = inactive_value(G);
    for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * blockDim.x)
        write_group(pool32 + gi * G.wb, G.wb, vals);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            st->t = 0;
            st->bact0 = 0;
        }
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) census_of(st)[d] = 0;
    }
}

// Census of group gi and its activity bitmap word: distances below k are
// counted into hist (LDS) when given, else into the census.
__device__ __forceinline__ void census_group_x(const Geo &G, const uint32_t *__restrict__ pool32, uint64_t gi,
                                               uint32_t bact0, uint32_t *hist, unsigned long long *census,
                                               uint8_t *__restrict__ bitmap)
{
    const uint32_t inact = inactive_value(G);
    uint32_t vals[32];
    read_group(pool32 + gi * G.wb, G.wb, vals);
    const uint64_t p0 = gi * 32;
    uint32_t bid0 = 0, act0 = 0;
    uint64_t next = 0;
    if (G.fast_blocks && !G.dr) {
        bid0 = block_of(G, (uint32_t)p0);
        act0 = block_act(G, bact0, bid0);
        next = block_start(G, bid0 + 1);
    }
    uint32_t bits = 0;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const uint32_t val = vals[e];
        if (val == inact) continue;
        uint32_t d;
        if (G.dr) {
            d = val;
        } else {
            uint32_t act;
            if (G.fast_blocks)
                act = p0 + e < next ? act0 : block_act(G, bact0, bid0 + 1);
            else
                act = block_act(G, bact0, block_of(G, (uint32_t)(p0 + e)));
            d = at_dist(G, act, val);
        }
        if (d < G.k) {
            bits |= 1u << e;
            if (hist) atomicAdd(&hist[d], 1u);
            else atomicAdd(&census[d], 1ull);
        }
    }
    reinterpret_cast<uint32_t *>(bitmap)[gi] = bits;
}

// Census and activity bitmap (one bitmap word per group).
__global__ void __launch_bounds__(256) k_census_x(Geo G, const uint32_t *__restrict__ pool32, uint64_t ngroups,
                                                  DevState *__restrict__ st, uint8_t *__restrict__ bitmap)
{
    __shared__ uint32_t hist[kCensusLdsBins];
    const bool lds = G.k <= kCensusLdsBins;
    if (lds)
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) hist[d] = 0;
    __syncthreads();
    const uint32_t bact0 = st->bact0;
    for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * blockDim.x)
        census_group_x(G, pool32, gi, bact0, lds ? hist : nullptr, census_of(st), bitmap);
    __syncthreads();
    if (lds)
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x)
            if (hist[d]) atomicAdd(&census_of(st)[d], (unsigned long long)hist[d]);
}

// Alg. 3 on the two blocks whose ACT is 0 or k; thread j < max_groups takes
// a group of the first block, the rest groups of the second (a group in both
// ranges is handled once, by the first).
__device__ __forceinline__ void preserve_group_x(const Geo &G, uint32_t *__restrict__ pool32, uint32_t bact0,
                                                 uint64_t j, uint64_t max_groups)
{
    const uint32_t i0 = bact0 == 0 ? 0 : G.twok - bact0;                        // (BACT^0 + i0) mod 2k == 0
    const uint32_t i1 = bact0 <= G.k ? G.k - bact0 : G.twok + G.k - bact0;      // == k
    const uint64_t s0 = block_start(G, i0), e0 = block_start(G, i0 + 1);
    const uint64_t s1 = block_start(G, i1), e1 = block_start(G, i1 + 1);
    const uint64_t g0lo = s0 / 32, g0hi = s0 < e0 ? (e0 + 31) / 32 : g0lo;
    const uint64_t g1lo = s1 / 32, g1hi = s1 < e1 ? (e1 + 31) / 32 : g1lo;
    if (j >= 2 * max_groups) return;
    const bool second = j >= max_groups;
    const uint64_t gi = second ? g1lo + (j - max_groups) : g0lo + j;
    if (gi >= (second ? g1hi : g0hi)) return;
    if (second && gi >= g0lo && gi < g0hi) return;
    uint32_t *words = pool32 + gi * G.wb;
    uint32_t vals[32];
    read_group(words, G.wb, vals);
    bool changed = false;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const uint64_t p = gi * 32 + e;
        const bool in0 = p >= s0 && p < e0, in1 = p >= s1 && p < e1;
        if (!in0 && !in1) continue;
        const uint32_t val = vals[e];
        bool mark;
        if (in0)   // ACT == 0: 0 <= Value <= k
            mark = val <= G.k;
        else       // ACT == k: k <= Value <= 2k-1, or Value == 0
            mark = (val >= G.k && val <= G.twok - 1) || val == 0;
        if (mark && val != G.twok) {
            vals[e] = G.twok;
            changed = true;
        }
    }
    if (changed) write_group(words, G.wb, vals);
}

__global__ void __launch_bounds__(256) k_preserve_x(Geo G, uint32_t *__restrict__ pool32,
                                                    const DevState *__restrict__ st, uint64_t max_groups)
{
    preserve_group_x(G, pool32, st->bact0, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, max_groups);
}

// DR maintenance: every counter of group gi grows by one, saturating at k.
__device__ __forceinline__ void dr_maintain_group_x(const Geo &G, uint32_t *__restrict__ pool32, uint64_t gi)
{
    uint32_t *words = pool32 + gi * G.wb;
    uint32_t vals[32];
    read_group(words, G.wb, vals);
    bool changed = false;
#pragma unroll
    for (int e = 0; e < 32; ++e)
        if (vals[e] < G.k) {
            ++vals[e];
            changed = true;
        }
    if (changed) write_group(words, G.wb, vals);
}

__global__ void __launch_bounds__(256) k_dr_maintain_x(Geo G, uint32_t *__restrict__ pool32, uint64_t ngroups)
{
    for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < ngroups;
         gi += (uint64_t)gridDim.x * blockDim.x)
        dr_maintain_group_x(G, pool32, gi);
}
