// Batched VATE: many independent sketches (different pools, widths, windows,
// packet counts and host lists) advanced through one time slice by one
// persistent launch per phase.  Included by vate.hip inside namespace vate.
//
// Every phase kernel is persistent: workgroups claim tiles from a per-phase
// counter until the phase's tiles (over all sketches, prefix-summed per
// sketch) are exhausted, so sketches with 1e5 and 1e7 packets share the chip
// without idle tails.  The per-slice tile tables are built on the device by
// k_batch_begin from the sketches' packet counts, so the whole slice can be
// captured once as a hipGraph and replayed.

constexpr uint32_t kBatchMax = 64;
constexpr uint32_t kBatchCensusBins = 4096;   // LDS histogram bins (k limit)

struct BatchItem {
    Geo G;
    uint8_t *pool;
    DevState *st;
    uint8_t *bitmap;
    const uint32_t *pairs;       // this slice's packets (fixed address)
    const uint32_t *hosts;
    float *est;
    uint32_t *live;
    uint64_t pairs_cap;          // capacity of the pair buffer (packets)
    uint64_t nchunks;            // streaming units: 16-byte pool chunks (exact widths: 32-counter groups)
    uint64_t max_block_chunks;   // units one due block can overlap
    uint32_t width, n_hosts, kprime, pad;   // width 0: an exact-width pool (G.wb bits per counter)
};

// Launch shape of each phase (chosen by the autotuner).
struct BatchTune {
    uint32_t ingest_tile;        // packets per claimed tile (multiple of 512)
    uint32_t census_tile;        // pool chunks per claimed tile (multiple of 256)
    uint32_t estimate_block;     // threads per estimate workgroup (64, 128 or 256)
    uint32_t grid_preserve, grid_ingest, grid_census, grid_estimate;
    uint32_t estimate_lanes;     // lanes per host (1, 4 or 16): hosts per tile = estimate_block / estimate_lanes
    uint32_t census_unroll;      // pool chunks in flight per census thread (1, 2 or 4)
};

enum { PH_PRESERVE = 0, PH_INGEST = 1, PH_CENSUS = 2, PH_ESTIMATE = 3, PH_COUNT = 4 };

struct BatchTables {
    unsigned long long prefix[PH_COUNT][kBatchMax + 1];
    unsigned int claim[PH_COUNT];
    unsigned int pad[PH_COUNT];
};

__device__ __forceinline__ uint32_t find_item(const unsigned long long *prefix, uint32_t S, unsigned long long tile)
{
    uint32_t lo = 0, hi = S;        // largest s < S with prefix[s] <= tile
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Claim the next tile of a phase for the whole workgroup.
__device__ __forceinline__ unsigned long long claim_tile(unsigned int *counter)
{
    __shared__ unsigned long long t;
    __syncthreads();
    if (threadIdx.x == 0) t = atomicAdd(counter, 1u);
    __syncthreads();
    return t;
}

// Start of a batch slice: advance the clocks of the sketches in adv_mask
// (Alg. 4 end of loop; census cleared), build the per-phase tile prefix
// tables from this slice's packet counts, reset the claim counters.
__global__ void k_batch_begin(BatchItem *__restrict__ items, uint32_t S, const unsigned long long *__restrict__ n_pairs,
                              unsigned long long adv_mask, BatchTune tune, BatchTables *__restrict__ tab)
{
    __shared__ unsigned long long tiles[PH_COUNT][kBatchMax];
    for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) {
        const BatchItem &it = items[s];
        if ((adv_mask >> s) & 1ull) {
            it.st->bact0 = it.st->bact0 + 1 == it.G.twok ? 0 : it.st->bact0 + 1;
            it.st->t = it.st->t + 1;
            // AT: the two due blocks; DR: the whole pool
            tiles[PH_PRESERVE][s] = it.G.dr ? (it.nchunks + 255) / 256 : (2 * it.max_block_chunks + 255) / 256;
        } else {
            tiles[PH_PRESERVE][s] = 0;
        }
        for (uint32_t d = 0; d < it.G.k; ++d) census_of(it.st)[d] = 0;
        const unsigned long long np = min((unsigned long long)n_pairs[s], (unsigned long long)it.pairs_cap);
        tiles[PH_INGEST][s] = (np + tune.ingest_tile - 1) / tune.ingest_tile;
        tiles[PH_CENSUS][s] = (it.nchunks + tune.census_tile - 1) / tune.census_tile;
        const uint32_t per_tile = tune.estimate_block / tune.estimate_lanes;
        tiles[PH_ESTIMATE][s] = ((unsigned long long)it.n_hosts + per_tile - 1) / per_tile;
    }
    __syncthreads();
    if (threadIdx.x < PH_COUNT) {
        const uint32_t ph = threadIdx.x;
        unsigned long long run = 0;
        for (uint32_t s = 0; s < S; ++s) {
            tab->prefix[ph][s] = run;
            run += tiles[ph][s];
        }
        tab->prefix[ph][S] = run;
        tab->claim[ph] = 0;
    }
}

__global__ void k_batch_reset_claim(BatchTables *__restrict__ tab, uint32_t ph)
{
    if (threadIdx.x == 0) tab->claim[ph] = 0;
}

__global__ void k_batch_clear_census(BatchItem *__restrict__ items, uint32_t S)
{
    for (uint32_t s = blockIdx.x; s < S; s += gridDim.x)
        for (uint32_t d = threadIdx.x; d < items[s].G.k; d += blockDim.x) census_of(items[s].st)[d] = 0;
}

__global__ void __launch_bounds__(256) k_batch_preserve(const BatchItem *__restrict__ items, uint32_t S,
                                                        BatchTables *__restrict__ tab)
{
    const unsigned long long total = tab->prefix[PH_PRESERVE][S];
    for (;;) {
        const unsigned long long tile = claim_tile(&tab->claim[PH_PRESERVE]);
        if (tile >= total) break;
        const uint32_t s = find_item(tab->prefix[PH_PRESERVE], S, tile);
        const BatchItem &it = items[s];
        const uint64_t j = (tile - tab->prefix[PH_PRESERVE][s]) * 256 + threadIdx.x;
        uint4 *pool4 = reinterpret_cast<uint4 *>(it.pool);
        uint32_t *pool32 = reinterpret_cast<uint32_t *>(it.pool);
        const uint32_t bact0 = it.st->bact0;
        if (it.G.dr) {
            if (j < it.nchunks) {
                if (it.width == 0) dr_maintain_group_x(it.G, pool32, j);
                else if (it.width == 4) dr_maintain_chunk<4>(it.G, pool4, j);
                else if (it.width == 8) dr_maintain_chunk<8>(it.G, pool4, j);
                else dr_maintain_chunk<16>(it.G, pool4, j);
            }
            continue;
        }
        if (it.width == 0) preserve_group_x(it.G, pool32, bact0, j, it.max_block_chunks);
        else if (it.width == 4) preserve_chunk<4>(it.G, pool4, bact0, j, it.max_block_chunks);
        else if (it.width == 8) preserve_chunk<8>(it.G, pool4, bact0, j, it.max_block_chunks);
        else preserve_chunk<16>(it.G, pool4, bact0, j, it.max_block_chunks);
    }
}

template <int W>
__device__ __forceinline__ void batch_ingest_tile(const BatchItem &it, uint64_t p0, uint64_t p1)
{
    const uint32_t bact0 = it.st->bact0;
    for (uint64_t j = p0 + 2ull * threadIdx.x; j < p1; j += 2ull * blockDim.x) {
        if (j + 2 <= p1) {
            const uint4 v = *reinterpret_cast<const uint4 *>(it.pairs + 2 * j);
            ingest_one<W>(it.G, it.pool, bact0, v.x, v.y);
            ingest_one<W>(it.G, it.pool, bact0, v.z, v.w);
        } else {
            const uint2 v = *reinterpret_cast<const uint2 *>(it.pairs + 2 * j);
            ingest_one<W>(it.G, it.pool, bact0, v.x, v.y);
        }
    }
}

// Packet tiles start at multiples of ingest_tile (even), so the 16-byte
// loads are aligned whenever the sketch's pair buffer is.
__global__ void __launch_bounds__(256) k_batch_ingest(const BatchItem *__restrict__ items, uint32_t S,
                                                      const unsigned long long *__restrict__ n_pairs, BatchTune tune,
                                                      BatchTables *__restrict__ tab)
{
    const unsigned long long total = tab->prefix[PH_INGEST][S];
    for (;;) {
        const unsigned long long tile = claim_tile(&tab->claim[PH_INGEST]);
        if (tile >= total) break;
        const uint32_t s = find_item(tab->prefix[PH_INGEST], S, tile);
        const BatchItem &it = items[s];
        const uint64_t p0 = (tile - tab->prefix[PH_INGEST][s]) * tune.ingest_tile;
        const uint64_t p1 = min(p0 + tune.ingest_tile, min((uint64_t)n_pairs[s], it.pairs_cap));
        if (it.width == 0) batch_ingest_tile<0>(it, p0, p1);
        else if (it.width == 4) batch_ingest_tile<4>(it, p0, p1);
        else if (it.width == 8) batch_ingest_tile<8>(it, p0, p1);
        else batch_ingest_tile<16>(it, p0, p1);
    }
}

template <int W, int U>
__device__ __forceinline__ void batch_census_tile(const BatchItem &it, uint64_t c0, uint64_t c1, uint32_t *hist)
{
    const uint32_t bact0 = it.st->bact0;
    const uint4 *pool4 = reinterpret_cast<const uint4 *>(it.pool);
    const uint32_t pat = replicate<W>(inactive_value(it.G));
    uint32_t *h = it.G.k <= kBatchCensusBins ? hist : nullptr;
    for (uint64_t b = c0 + threadIdx.x; b < c1; b += U * blockDim.x) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t ch = b + (uint64_t)u * blockDim.x;
            v[u] = ch < c1 ? pool4[ch] : make_uint4(pat, pat, pat, pat);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t ch = b + (uint64_t)u * blockDim.x;
            if (ch < c1) store_bits<W>(it.bitmap, ch, census_chunk_fast<W>(it.G, v[u], ch, bact0, pat, h, census_of(it.st)));
        }
    }
}

// Exact widths: groups [c0, c1) of 32 counters.
__device__ __forceinline__ void batch_census_groups(const BatchItem &it, uint64_t c0, uint64_t c1, uint32_t *hist)
{
    const uint32_t bact0 = it.st->bact0;
    const uint32_t *pool32 = reinterpret_cast<const uint32_t *>(it.pool);
    uint32_t *h = it.G.k <= kBatchCensusBins ? hist : nullptr;
    for (uint64_t gi = c0 + threadIdx.x; gi < c1; gi += blockDim.x)
        census_group_x(it.G, pool32, gi, bact0, h, census_of(it.st), it.bitmap);
}

// The LDS histogram belongs to one sketch at a time: it is flushed into that
// sketch's census when the claimed tiles move on to another sketch.
template <int U>
__global__ void __launch_bounds__(256) k_batch_census(const BatchItem *__restrict__ items, uint32_t S, BatchTune tune,
                                                      BatchTables *__restrict__ tab)
{
    __shared__ uint32_t hist[kBatchCensusBins];
    const unsigned long long total = tab->prefix[PH_CENSUS][S];
    int cur = -1;
    for (;;) {
        const unsigned long long tile = claim_tile(&tab->claim[PH_CENSUS]);
        const int s = tile >= total ? -2 : (int)find_item(tab->prefix[PH_CENSUS], S, tile);
        if (s != cur) {
            if (cur >= 0 && items[cur].G.k <= kBatchCensusBins)
                for (uint32_t d = threadIdx.x; d < items[cur].G.k; d += blockDim.x)
                    if (hist[d]) atomicAdd(&census_of(items[cur].st)[d], (unsigned long long)hist[d]);
            __syncthreads();
            if (s >= 0)
                for (uint32_t d = threadIdx.x; d < min(items[s].G.k, kBatchCensusBins); d += blockDim.x) hist[d] = 0;
            __syncthreads();
            cur = s;
        }
        if (s < 0) break;
        const BatchItem &it = items[s];
        const uint64_t c0 = (tile - tab->prefix[PH_CENSUS][s]) * tune.census_tile;
        const uint64_t c1 = min(c0 + tune.census_tile, it.nchunks);
        if (it.width == 0) batch_census_groups(it, c0, c1, hist);
        else if (it.width == 4) batch_census_tile<4, U>(it, c0, c1, hist);
        else if (it.width == 8) batch_census_tile<8, U>(it, c0, c1, hist);
        else batch_census_tile<16, U>(it, c0, c1, hist);
    }
}

// Live VATs of one host counted by L lanes: lane `sub` of the host's L takes
// VATs sub, sub + L, ... (kEstU gathers in flight), and the L partial counts
// are summed across the lanes (every lane of the wavefront takes part).
template <int W, int L>
__device__ __forceinline__ uint32_t batch_host_live(const BatchItem &it, uint32_t key, bool valid, uint32_t bact0,
                                                    uint32_t sub)
{
    const Geo &G = it.G;
    const bool need_dist = it.kprime < G.k;
    uint32_t live = 0;
    for (uint32_t i0 = sub; i0 < G.g; i0 += L * kEstU) {
        uint32_t pid[kEstU], byte[kEstU];
#pragma unroll
        for (int u = 0; u < kEstU; ++u) pid[u] = vat_pid(G, key, i0 + u * L);
#pragma unroll
        for (int u = 0; u < kEstU; ++u) byte[u] = (valid && i0 + u * L < G.g) ? it.bitmap[pid[u] >> 3] : 0u;
#pragma unroll
        for (int u = 0; u < kEstU; ++u) {
            if (!((byte[u] >> (pid[u] & 7u)) & 1u)) continue;
            if (!need_dist) {
                ++live;
                continue;
            }
            const uint32_t d = value_dist(G, bact0, pid[u], load_at<W>(it.pool, pid[u], it.G.wb));
            live += d < it.kprime;
        }
    }
#pragma unroll
    for (int off = 1; off < L; off <<= 1) live += __shfl_xor(live, off, 64);
    return live;
}

template <int L>
__global__ void __launch_bounds__(256) k_batch_estimate(const BatchItem *__restrict__ items, uint32_t S,
                                                        BatchTune tune, BatchTables *__restrict__ tab)
{
    const unsigned long long total = tab->prefix[PH_ESTIMATE][S];
    const uint32_t per_tile = blockDim.x / L, sub = threadIdx.x % L;
    for (;;) {
        const unsigned long long tile = claim_tile(&tab->claim[PH_ESTIMATE]);
        if (tile >= total) break;
        const uint32_t s = find_item(tab->prefix[PH_ESTIMATE], S, tile);
        const BatchItem &it = items[s];
        const uint64_t active_pool = pool_active(it.st, it.kprime);
        const uint32_t bact0 = it.st->bact0;
        const uint64_t h = (tile - tab->prefix[PH_ESTIMATE][s]) * per_tile + threadIdx.x / L;
        const bool valid = h < it.n_hosts;
        const uint32_t key = host_key(it.G, valid ? it.hosts[h] : 0u);
        uint32_t live;
        if (it.width == 0) live = batch_host_live<0, L>(it, key, valid, bact0, sub);
        else if (it.width == 4) live = batch_host_live<4, L>(it, key, valid, bact0, sub);
        else if (it.width == 8) live = batch_host_live<8, L>(it, key, valid, bact0, sub);
        else live = batch_host_live<16, L>(it, key, valid, bact0, sub);
        if (valid && sub == 0) {
            it.est[h] = estimate_from_counts(it.G.g - live, it.G.N - active_pool, it.G.g, it.G.c);
            if (it.live) it.live[h] = live;
        }
    }
}
