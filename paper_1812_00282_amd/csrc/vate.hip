// VATE hot path for MI355X (gfx950): pool init, packet ingest (SetAT),
// pool census, per-host estimation, clock advance and two-block preservation,
// behind the C ABI declared in include/vate.h.
//
// Paper: Xu, Ding, Hu, "VATE: a trade-off between memory and preserving time
// for high accuracy cardinalities estimation under sliding time window",
// arXiv 1812.00282.  Algorithm 4 is the per-slice loop; Sec. 4.2 describes
// its three GPU phases (scan, estimate, maintain), which map to
// k_ingest, k_census + k_estimate and k_advance + k_preserve here.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "vate.h"
#include "vate_core.h"
#include "vate_mlp.h"
#include "mlp_core.h"
#include "vate_batch.h"

namespace vate {

// ---------------------------------------------------------------------------
// Device state block (caller-owned, 256-byte aligned).
// ---------------------------------------------------------------------------
struct DevState {
    unsigned long long t;        // current slice
    uint32_t bact0;              // ACT of block 0 (Eq. 7)
    uint32_t pad0;
    unsigned long long pad1[2];
};
constexpr size_t kStateHeader = sizeof(DevState);
static_assert(kStateHeader == 32, "state header layout");

// k counters follow the header: pool ATs whose distance is d < k.
__host__ __device__ __forceinline__ unsigned long long *census_of(DevState *st)
{
    return reinterpret_cast<unsigned long long *>(st + 1);
}
__host__ __device__ __forceinline__ const unsigned long long *census_of(const DevState *st)
{
    return reinterpret_cast<const unsigned long long *>(st + 1);
}
constexpr int kMaxHistK = 256;
constexpr uint32_t kCensusLdsBins = 4096;   // census histogram bins kept in LDS      // per-host histogram limit (LDS budget)

// State block layout: header, k census counters, then (256-byte aligned) the
// activity bitmap of N bits.
static size_t bitmap_offset(uint32_t k)
{
    size_t b = kStateHeader + 8ull * k;
    return (b + 255) & ~size_t(255);
}

static size_t bitmap_bytes(uint64_t N)
{
    size_t bm = (size_t)((N + 7) / 8);
    return bm < 16 ? 16 : bm;
}

// After the bitmap: kCensusCopies partial censuses (k counters each) that
// k_census8's workgroups add into, so that no counter takes an atomic from
// every workgroup; k_census_fold then adds them to the census and clears
// them (they are zero between censuses).
constexpr uint32_t kCensusCopies = 16;

static size_t copies_offset(uint32_t k, uint64_t N)
{
    return (bitmap_offset(k) + bitmap_bytes(N) + 255) & ~size_t(255);
}

static size_t state_bytes_for(uint32_t k, uint64_t N)
{
    return (copies_offset(k, N) + 8ull * kCensusCopies * k + 255) & ~size_t(255);
}

// ---------------------------------------------------------------------------
// Parameter validation / geometry.
// ---------------------------------------------------------------------------
int make_geo(const vate_params *p, Geo *G, const char **why)
{
    if (!p) { *why = "params is NULL"; return VATE_E_INVAL; }
    if (p->counter > 1) { *why = "counter must be 0 (AT) or 1 (DR)"; return VATE_E_INVAL; }
    if (p->log2_pool < 1 || p->log2_pool > 32) { *why = "log2_pool must be in [1, 32]"; return VATE_E_INVAL; }
    if (p->width < 1 || p->width > 16) { *why = "width must be in [1, 16]"; return VATE_E_INVAL; }
    if (p->k < 1) { *why = "k must be >= 1"; return VATE_E_INVAL; }
    if (p->counter == 0 && (1ull << p->width) < 2ull * p->k + 1) {
        *why = "width too small: an AT needs 2^width >= 2k+1";
        return VATE_E_INVAL;
    }
    if (p->counter == 1 && (1ull << p->width) < 1ull * p->k + 1) {
        *why = "width too small: a DR needs 2^width >= k+1";
        return VATE_E_INVAL;
    }
    if (p->g < 1 || p->g > 65535) { *why = "g must be in [1, 65535]"; return VATE_E_INVAL; }
    if (p->partition > 1) { *why = "partition must be 0 or 1"; return VATE_E_INVAL; }
    if (p->block_log2 > 10 || p->block_log2 > p->log2_pool) {
        *why = "block_log2 must be in [0, min(10, log2_pool)]";
        return VATE_E_INVAL;
    }
    uint64_t N = 1ull << p->log2_pool;
    if (N < 2ull * p->k) { *why = "pool smaller than 2k ATs"; return VATE_E_INVAL; }
    const bool exact = p->width != 4 && p->width != 8 && p->width != 16;
    if (!exact && N * p->width / 8 < 16) { *why = "pool smaller than 16 bytes"; return VATE_E_INVAL; }
    if (exact && N < 32) { *why = "widths other than 4, 8, 16 need a pool of >= 32 counters"; return VATE_E_INVAL; }
    Geo g{};
    g.N = N;
    g.c = p->log2_pool;
    g.shift = 32 - p->log2_pool;
    g.k = p->k;
    g.twok = 2 * p->k;
    g.g = p->g;
    g.seed_a = p->seed_a;
    g.seed_b = p->seed_b;
    g.partition = p->partition;
    g.dr = p->counter;
    g.wb = p->width;
    g.blog = p->block_log2;
    const uint64_t E = exact ? 32 : 128 / p->width;   // counters per 16-byte chunk / per word group
    if (p->partition == 0) {
        g.a = N / (g.twok - 1);
        g.thresh = 0;
        g.base1 = 0;
        g.div_a = make_div32(g.a);
        g.div_a1 = make_div32(1);
        g.fast_blocks = g.a >= E;
    } else {
        uint64_t ap = N / g.twok, bp = N % g.twok;
        g.a = ap;
        g.base1 = (uint32_t)(g.twok - bp);
        g.thresh = ap * (g.twok - bp);
        g.div_a = make_div32(ap);
        g.div_a1 = make_div32(ap + 1);
        g.fast_blocks = ap >= E;
    }
    *G = g;
    *why = "";
    return VATE_OK;
}

// ---------------------------------------------------------------------------
// Container access.  AT p sits at bits [p*W, p*W+W) of the pool, little-endian.
// ---------------------------------------------------------------------------
#include "vate_exact.h"

// W = 0: the exact width wb (counters packed back to back in 32-bit words).
template <int W>
__device__ __forceinline__ uint32_t load_at(const uint8_t *__restrict__ pool, uint32_t pid, uint32_t wb)
{
    if constexpr (W == 0) {
        return load_x(reinterpret_cast<const uint32_t *>(pool), pid, wb);
    } else if constexpr (W == 8) {
        return pool[pid];
    } else if constexpr (W == 16) {
        return reinterpret_cast<const uint16_t *>(pool)[pid];
    } else {
        return (pool[pid >> 1] >> ((pid & 1u) << 2)) & 0xFu;
    }
}

// Value e (0 <= e < 128/W) of a 16-byte chunk.
template <int W>
__device__ __forceinline__ uint32_t chunk_get(const uint4 &v, uint32_t e)
{
    constexpr uint32_t per_word = 32 / W;
    uint32_t w = e / per_word, s = (e % per_word) * W;
    uint32_t word = w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
    return (word >> s) & ((1u << W) - 1u);
}

template <int W>
__device__ __forceinline__ void chunk_set(uint4 &v, uint32_t e, uint32_t val)
{
    constexpr uint32_t per_word = 32 / W;
    uint32_t w = e / per_word, s = (e % per_word) * W;
    uint32_t mask = ((1u << W) - 1u) << s;
    uint32_t *word = w == 0 ? &v.x : w == 1 ? &v.y : w == 2 ? &v.z : &v.w;
    *word = (*word & ~mask) | (val << s);
}

template <int W>
__host__ __device__ __forceinline__ uint32_t replicate(uint32_t val)
{
    uint32_t r = 0;
    for (int s = 0; s < 32; s += W) r |= val << s;
    return r;
}

// ---------------------------------------------------------------------------
// k_init: InitAT on every AT (value 2k), t = 0, BACT^0 = 0, census cleared.
// ---------------------------------------------------------------------------
template <int W>
__global__ void __launch_bounds__(256) k_init(Geo G, uint4 *__restrict__ pool4, uint64_t nchunks,
                                              DevState *__restrict__ st, unsigned long long *__restrict__ copies)
{
    const uint32_t pat = replicate<W>(inactive_value(G));
    const uint4 v = make_uint4(pat, pat, pat, pat);
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < nchunks; i += (uint64_t)gridDim.x * blockDim.x) pool4[i] = v;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            st->t = 0;
            st->bact0 = 0;
        }
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) census_of(st)[d] = 0;
        for (uint32_t d = threadIdx.x; d < kCensusCopies * G.k; d += blockDim.x) copies[d] = 0;
    }
}

// ---------------------------------------------------------------------------
// k_ingest: the scan phase.  Each thread takes 4 consecutive packets (two
// 16-byte loads, so a wavefront reads 2 x 1 KiB contiguous), hashes them in
// registers and stores the block ACT into the AT (SetAT).  Concurrent SetATs
// of one AT in a slice all write the same value, so plain byte/short stores
// are race-free; 4-bit ATs share a 32-bit word with a neighbour and are
// written with an atomic OR of the set bits then an atomic AND of the clear
// bits, which leaves the nibble equal to ACT whatever the interleaving.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void set_at(uint8_t *__restrict__ pool, uint32_t pid, uint32_t act)
{
    if constexpr (W == 8) {
        pool[pid] = (uint8_t)act;
    } else if constexpr (W == 16) {
        reinterpret_cast<uint16_t *>(pool)[pid] = (uint16_t)act;
    } else {
        uint32_t *w32 = reinterpret_cast<uint32_t *>(pool) + (pid >> 3);
        uint32_t s = (pid & 7u) << 2;
        atomicOr(w32, act << s);
        atomicAnd(w32, ~((~act & 0xFu) << s));
    }
}

template <int W>
__device__ __forceinline__ void ingest_one(const Geo &G, uint8_t *__restrict__ pool, uint32_t bact0,
                                           uint32_t aip, uint32_t bip)
{
    uint32_t vid = bh(G, bip);
    uint32_t pid = vat_pid(G, host_key(G, aip), vid);
    // SetAT stores the block's ACT; a DR is reset to 0
    uint32_t val = G.dr ? 0u : block_act(G, bact0, block_of(G, pid));
    if constexpr (W == 0)
        set_x(reinterpret_cast<uint32_t *>(pool), pid, G.wb, val);
    else
        set_at<W>(pool, pid, val);
}

template <int W, bool ALIGNED16>
__global__ void __launch_bounds__(256) k_ingest(Geo G, const uint32_t *__restrict__ pairs, uint64_t n,
                                                uint8_t *__restrict__ pool, const DevState *__restrict__ st)
{
    const uint32_t bact0 = st->bact0;
    const uint64_t base = (uint64_t)blockIdx.x * 1024;   // packets per block
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const uint64_t j = base + (uint64_t)half * 512 + 2ull * threadIdx.x;   // first of 2 packets
        if (ALIGNED16 && j + 2 <= n) {
            uint4 v = reinterpret_cast<const uint4 *>(pairs)[j >> 1];
            ingest_one<W>(G, pool, bact0, v.x, v.y);
            ingest_one<W>(G, pool, bact0, v.z, v.w);
        } else {
            for (uint64_t q = j; q < j + 2 && q < n; ++q) {
                uint2 v = reinterpret_cast<const uint2 *>(pairs)[q];
                ingest_one<W>(G, pool, bact0, v.x, v.y);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_census: one streaming pass over the pool at the end of a slice.  Builds
// the histogram of AT distances d < k (Eq. 5) with per-workgroup LDS counters
// flushed by 64-bit atomics; Z_p for any k' is then N minus a prefix sum.
// In steady state most ATs hold 2k, so 16-byte chunks that are entirely
// inactive are skipped after one compare.
// ---------------------------------------------------------------------------

// The same pass writes the activity bitmap: bit p is set iff AT p is active
// for the longest window k at the end of this slice (value != 2k and
// distance < k).  The bitmap (N bits; 32 MiB for 2^28 ATs) is small enough to
// stay resident in the MI355X's 256 MB Infinity Cache, so the per-host gather
// in k_estimate reads bits from it instead of AT bytes from HBM.
template <int W>
__device__ __forceinline__ void store_bits(uint8_t *__restrict__ bitmap, uint64_t ch, uint32_t bits)
{
    if constexpr (W == 8)
        reinterpret_cast<uint16_t *>(bitmap)[ch] = (uint16_t)bits;   // 16 ATs per chunk
    else if constexpr (W == 4)
        reinterpret_cast<uint32_t *>(bitmap)[ch] = bits;             // 32 ATs per chunk
    else
        bitmap[ch] = (uint8_t)bits;                                  // 8 ATs per chunk
}

// One 16-byte chunk of the census: returns the chunk's activity bits and adds
// each active AT's distance to hist (LDS counters) or, without LDS, directly
// to the sketch's census.
template <int W>
__device__ __forceinline__ uint32_t census_chunk(const Geo &G, const uint4 &v, uint64_t ch, uint32_t bact0,
                                                 uint32_t *hist, unsigned long long *census)
{
    constexpr uint32_t E = 128 / W;
    const uint32_t inact = inactive_value(G);
    const uint32_t pat = replicate<W>(inact);
    if (v.x == pat && v.y == pat && v.z == pat && v.w == pat) return 0;
    uint32_t bits = 0;
    const uint64_t p0 = ch * E;
    uint32_t bid0 = 0, act0 = 0;
    uint64_t next = 0;
    if (G.fast_blocks && !G.dr) {
        bid0 = block_of(G, (uint32_t)p0);
        act0 = block_act(G, bact0, bid0);
        next = block_start(G, bid0 + 1);
    }
    for (uint32_t e = 0; e < E; ++e) {
        uint32_t val = chunk_get<W>(v, e);
        if (val == inact) continue;
        uint32_t d;
        if (G.dr) {
            d = val;                         // a DR holds its distance
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
    return bits;
}

// Byte ATs of a chunk inside one block: the activity test four ATs at a time
// in packed 16-bit lanes (each 32-bit word split into its even and odd
// bytes).  For ACT a and value v in [0, 2k]: u = a + 2k - v, the distance is
// (a - v) mod 2k = min(u, u - 2k) (the second wraps when u < 2k), raised to
// at least k when v = 2k (inactive), and the AT is active iff it is below k.
// A DR's value is its distance.  Only the active ATs (a few per cent) take
// the per-AT histogram step.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t active_bits8(const Geo &G, const uint4 &v, uint32_t act)
{
    const u16x2 K = (u16x2)(unsigned short)G.k;
    const u16x2 A = (u16x2)(unsigned short)(act + G.twok);
    const u16x2 T = (u16x2)(unsigned short)G.twok;
    const u16x2 T1 = (u16x2)(unsigned short)(G.twok - 1u);
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t f2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u16x2 x = __builtin_bit_cast(u16x2, (w4[j] >> (8 * h)) & 0x00FF00FFu);
            u16x2 d;
            if (G.dr) {
                d = x;
            } else {
                const u16x2 u = A - x;
                d = __builtin_elementwise_min(u, u - T);
                d = __builtin_elementwise_max(d, __builtin_elementwise_sub_sat(x, T1) * K);
            }
            f2[h] = __builtin_bit_cast(uint32_t, (u16x2)((d - K) >> (unsigned short)15));   // 1 iff d < k
        }
        // f2[0] holds bytes 0 and 2 of word j, f2[1] bytes 1 and 3
        const uint32_t x = f2[0] | (f2[1] << 1);
        bits |= ((x & 3u) | ((x >> 14) & 0xCu)) << (4 * j);
    }
    return bits;
}

// One chunk of the census with the fast paths: an all-inactive chunk (most
// of them in steady state) has no bits; byte ATs of a chunk inside one block
// (or any chunk of byte DRs) take the packed test when the histogram is in
// LDS; anything else goes through census_chunk.
template <int W>
__device__ __forceinline__ uint32_t census_chunk_fast(const Geo &G, const uint4 &v, uint64_t ch, uint32_t bact0,
                                                      uint32_t pat, uint32_t *hist, unsigned long long *census)
{
    if constexpr (W == 8) {
        if (v.x == pat && v.y == pat && v.z == pat && v.w == pat) return 0u;
        if (hist) {
            const uint32_t p0 = (uint32_t)(ch * 16u);
            uint32_t bid0 = 0, act = 0;
            bool one = G.dr != 0;
            if (!one && G.fast_blocks) {
                bid0 = block_of(G, p0);
                one = (uint64_t)p0 + 16u <= block_start(G, bid0 + 1);
                act = block_act(G, bact0, bid0);
            }
            if (one) {
                const uint32_t bits = active_bits8(G, v, act);
                uint32_t rest = bits;
                while (rest) {
                    const uint32_t e = __builtin_ctz(rest);
                    rest &= rest - 1u;
                    const uint32_t val = chunk_get<8>(v, e);
                    atomicAdd(&hist[G.dr ? val : at_dist(G, act, val)], 1u);
                }
                return bits;
            }
        }
    }
    return census_chunk<W>(G, v, ch, bact0, hist, census);
}

template <int W>
__global__ void __launch_bounds__(256) k_census(Geo G, const uint4 *__restrict__ pool4, uint64_t nchunks,
                                                DevState *__restrict__ st, uint8_t *__restrict__ bitmap)
{
    __shared__ uint32_t hist[kCensusLdsBins];
    const bool lds = G.k <= kCensusLdsBins;
    if (lds)
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) hist[d] = 0;
    __syncthreads();
    const uint32_t bact0 = st->bact0;
    const uint32_t pat = replicate<W>(inactive_value(G));
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c0 < nchunks; c0 += U * stride) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint64_t ch = c0 + u * stride;
            v[u] = ch < nchunks ? pool4[ch] : make_uint4(pat, pat, pat, pat);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t ch = c0 + u * stride;
            if (ch < nchunks)
                store_bits<W>(bitmap, ch,
                              census_chunk_fast<W>(G, v[u], ch, bact0, pat, lds ? hist : nullptr, census_of(st)));
        }
    }
    __syncthreads();
    if (lds)
        for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x)
            if (hist[d]) atomicAdd(&census_of(st)[d], (unsigned long long)hist[d]);
}

// k_census8: the census of byte counters with k <= kCensus8Bins.  In steady
// state only a few per cent of the chunks hold an active AT, but nearly every
// wavefront has one among its 64, so a per-lane test would run the packed
// activity test on all of them.  Here each wavefront stages the busy chunks
// of a round in LDS (compacted, in lane order), its lanes test the staged
// chunks one each and leave each chunk's bits in its staging slot, and the
// chunk's own lane picks them up; all-inactive chunks have zero bits.
//
// A lane takes U consecutive chunks per round (64 contiguous bytes, a
// wavefront 4 KiB) and stores their 16-bit bitmap words as one 8-byte
// store.  The rounds in which every lane's chunks lie inside the pool are
// software pipelined: a round's loads are issued before the previous round
// is tested, and its bitmap store after, so the wait for the loads never
// covers a store that is still in flight.  The remaining round (at most
// one) is guarded.
constexpr uint32_t kCensus8Bins = 256;
constexpr int kCensus8U = 4;   // consecutive chunks per lane and round

struct Census8Lds {
    uint32_t hist[kCensus8Bins];
    uint4 v[4][64 * kCensus8U];       // staged chunks of each wavefront
    uint16_t c[4][64 * kCensus8U];    // staged chunk's (u * 64 + lane), then its bits
};

// One round: chunk u of this lane is c0 + u; bits[u] = its activity bits.
__device__ __forceinline__ void census8_round(const Geo &G, const uint4 (&v)[kCensus8U], uint64_t c0, uint32_t bact0,
                                              uint32_t pat, Census8Lds &L, uint32_t (&bits)[kCensus8U],
                                              unsigned long long *census)
{
    constexpr int U = kCensus8U;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t n = 0;          // staged chunks of this wavefront (uniform)
    uint32_t pos[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool busy = v[u].x != pat || v[u].y != pat || v[u].z != pat || v[u].w != pat;
        const uint64_t m = __ballot(busy);
        pos[u] = busy ? n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull)) : ~0u;
        if (busy) {
            L.v[wv][pos[u]] = v[u];
            L.c[wv][pos[u]] = (uint16_t)(u * 64 + lane);
        }
        n += (uint32_t)__popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t wbase = c0 - (uint64_t)U * lane;     // the wavefront's first chunk
    for (uint32_t i = lane; i < n; i += 64) {
        const uint32_t code = L.c[wv][i];
        const uint64_t ch = wbase + (uint64_t)U * (code & 63u) + (code >> 6);
        L.c[wv][i] = (uint16_t)census_chunk_fast<8>(G, L.v[wv][i], ch, bact0, pat, L.hist, census);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int u = 0; u < U; ++u) bits[u] = pos[u] != ~0u ? (uint32_t)L.c[wv][pos[u]] : 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256) k_census8(Geo G, const uint4 *__restrict__ pool4, uint64_t nchunks,
                                                 DevState *__restrict__ st, uint8_t *__restrict__ bitmap,
                                                 unsigned long long *__restrict__ copies)
{
    constexpr int U = kCensus8U;
    static_assert(U == 4, "one 8-byte bitmap store per lane and round");
    __shared__ Census8Lds L;
    for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) L.hist[d] = 0;
    __syncthreads();
    const uint32_t bact0 = st->bact0;
    const uint32_t pat = replicate<8>(inactive_value(G));
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t step = (uint64_t)U * gridDim.x * blockDim.x;     // chunks per round
    uint16_t *bm16 = reinterpret_cast<uint16_t *>(bitmap);
    uint64_t c0 = (uint64_t)U * (blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t bits[U];
    const uint64_t full = nchunks / step;      // rounds with every chunk inside the pool
    if (full > 0) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = pool4[c0 + u];
        // The first round's chunks are waited for here, so that the loop
        // entry leaves no load in flight that the loop head would wait for
        // (a wait there would also cover the previous round's store).
#pragma unroll
        for (int u = 0; u < U; ++u) asm volatile("" ::"v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w));
        for (uint64_t r = 0; r < full; ++r, c0 += step) {
            // the next round's chunks (the last round reloads its own)
            const uint64_t nx = r + 1 < full ? c0 + step : c0;
            uint4 w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = pool4[nx + u];
            census8_round(G, v, c0, bact0, pat, L, bits, census_of(st));
            *reinterpret_cast<uint2 *>(bm16 + c0) = make_uint2(bits[0] | bits[1] << 16, bits[2] | bits[3] << 16);
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = w[u];
        }
    }
    if (c0 - (uint64_t)U * lane < nchunks) {   // the guarded last round (uniform per wavefront)
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = c0 + u < nchunks ? pool4[c0 + u] : make_uint4(pat, pat, pat, pat);
        census8_round(G, v, c0, bact0, pat, L, bits, census_of(st));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c0 + u < nchunks) bm16[c0 + u] = (uint16_t)bits[u];
    }
    __syncthreads();
    // Flush into copy blockIdx mod kCensusCopies (k_census_fold adds the
    // copies to the census).
    unsigned long long *mine = copies + (size_t)(blockIdx.x % kCensusCopies) * G.k;
    for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x)
        if (L.hist[d]) atomicAdd(&mine[d], (unsigned long long)L.hist[d]);
}

__global__ void __launch_bounds__(256) k_census_fold(Geo G, DevState *__restrict__ st,
                                                     unsigned long long *__restrict__ copies)
{
    for (uint32_t d = blockIdx.x * blockDim.x + threadIdx.x; d < G.k; d += gridDim.x * blockDim.x) {
        unsigned long long sum = 0;
        for (uint32_t c = 0; c < kCensusCopies; ++c) {
            sum += copies[(size_t)c * G.k + d];
            copies[(size_t)c * G.k + d] = 0;
        }
        census_of(st)[d] += sum;
    }
}

// ---------------------------------------------------------------------------
// k_estimate: one thread per host.  The g VATs of the host are gathered in
// batches of U independent byte loads (U gathers of 64 random lines in flight
// per wavefront), decoded with CheckAT (Alg. 1), counted, and the estimate
// of Eq. 11 is formed in FP32 from exact integer counts.  With HIST each
// lane also keeps the host's distance histogram in LDS as pairs of 16-bit
// counters in lane-private columns (conflict-free increments), written out
// transposed so that the (hosts x (k+1)) output is stored contiguously.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float estimate_from_counts(uint64_t u_v, uint64_t u_p, uint32_t g, uint32_t c)
{
    if (u_v == 0) u_v = 1;
    if (u_p == 0) u_p = 1;
    const uint64_t N = 1ull << c;
    const long long D = (long long)(u_p * g) - (long long)(N * u_v);
    const float den = ldexpf((float)u_v, (int)c);          // N * u_v, exact
    const float x = (float)D / den;
    if (x >= -0.5f)
        return (float)g * log1pf(x);
    return (float)g * logf((float)(u_p * g) / den);
}

// Number of pool ATs active for k' (sum of census bins d < k'), per wavefront.
__device__ __forceinline__ uint64_t pool_active(const DevState *__restrict__ st, uint32_t kprime)
{
    const uint32_t lane = threadIdx.x & 63u;
    unsigned long long s = 0;
    for (uint32_t d = lane; d < kprime; d += 64) s += census_of(st)[d];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

constexpr int kEstU = 16;   // VAT gathers in flight per thread

template <int W, bool HIST>
__global__ void __launch_bounds__(256) k_estimate(Geo G, const uint8_t *__restrict__ pool,
                                                  const DevState *__restrict__ st,
                                                  const uint8_t *__restrict__ bitmap,
                                                  const uint32_t *__restrict__ hosts, uint32_t n,
                                                  uint32_t kprime, float *__restrict__ est,
                                                  uint32_t *__restrict__ live_out,
                                                  uint32_t *__restrict__ hist_out)
{
    extern __shared__ uint32_t lds_hist[];   // HIST: [waves][rows + 1][65]
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t rows = (G.k + 1) / 2;     // bins d and d^1 share a dword
    uint32_t *my = lds_hist + (size_t)wave * (rows + 1) * 65;
    if (HIST) {
        for (uint32_t r = 0; r < rows; ++r) my[r * 65 + lane] = 0;
    }
    const uint64_t active_pool = pool_active(st, kprime);
    const uint32_t bact0 = st->bact0;
    // The bitmap answers CheckAT(., k) directly; the AT value (for its
    // distance) is only fetched for VATs that are active at all, and only
    // when a shorter window or the histogram needs it.
    const bool need_dist = HIST || kprime < G.k;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = h < n;
    const uint32_t key = host_key(G, valid ? hosts[h] : 0u);
    uint32_t live = 0, live_k = 0;
    for (uint32_t i0 = 0; i0 < G.g; i0 += kEstU) {
        uint32_t pid[kEstU], byte[kEstU];
#pragma unroll
        for (int u = 0; u < kEstU; ++u) pid[u] = vat_pid(G, key, i0 + u);
#pragma unroll
        for (int u = 0; u < kEstU; ++u)
            byte[u] = (valid && i0 + u < G.g) ? bitmap[pid[u] >> 3] : 0u;
#pragma unroll
        for (int u = 0; u < kEstU; ++u) {
            if (!((byte[u] >> (pid[u] & 7u)) & 1u)) continue;
            if (!need_dist) {
                ++live;
                continue;
            }
            const uint32_t d = value_dist(G, bact0, pid[u], load_at<W>(pool, pid[u], G.wb));
            live += d < kprime;
            if (HIST) {
                ++live_k;
                atomicAdd(&my[(d >> 1) * 65 + lane], 1u << ((d & 1u) << 4));
            }
        }
    }
    if (valid) {
        est[h] = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
        if (live_out) live_out[h] = live;
    }
    if (HIST) {
        my[rows * 65 + lane] = live_k;
        __syncthreads();
        const uint32_t h0 = blockIdx.x * blockDim.x + wave * 64;
        if (h0 < n) {
            const uint32_t nh = min(64u, n - h0), kp1 = G.k + 1;
            uint32_t *out = hist_out + (size_t)h0 * kp1;
            for (uint32_t e = lane; e < nh * kp1; e += 64) {
                const uint32_t host = e / kp1, bin = e - host * kp1;
                uint32_t v;
                if (bin < G.k)
                    v = (my[(bin >> 1) * 65 + host] >> ((bin & 1u) << 4)) & 0xFFFFu;
                else
                    v = G.g - my[rows * 65 + host];
                out[e] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_estimate_blocked: the closed form for window k under the locality-blocked
// H with blocks of >= 32 VATs, where a block is whole 32-bit words of the
// activity bitmap.  L lanes per host (L = blocks per host rounded up to a
// power of two, at most 64), each counting the set bits of its blocks with
// popcount; the host's lanes are summed by shuffles.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_estimate_blocked(Geo G, const DevState *__restrict__ st,
                                                          const uint32_t *__restrict__ bitmap,
                                                          const uint32_t *__restrict__ hosts, uint32_t n,
                                                          uint32_t lanes_log2, float *__restrict__ est,
                                                          uint32_t *__restrict__ live_out)
{
    const uint64_t active_pool = pool_active(st, G.k);
    const uint32_t L = 1u << lanes_log2;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t h = gid >> lanes_log2, sub = gid & (L - 1u);
    const bool valid = h < n;
    const uint32_t key = host_key(G, valid ? hosts[h] : 0u);
    const uint32_t beta = 1u << G.blog, words = beta >> 5;
    const uint32_t nb = (G.g + beta - 1u) >> G.blog;
    uint32_t live = 0;
    if (valid)
        for (uint32_t q = sub; q < nb; q += L) {
            const uint32_t base = vat_pid(G, key, q << G.blog);          // block-aligned first AT
            const uint32_t in_block = min(beta, G.g - (q << G.blog));      // VATs of this block
            const uint32_t *w = bitmap + (base >> 5);
            for (uint32_t x = 0; x < words; ++x) {
                const uint32_t lo = x << 5;
                if (lo >= in_block) break;
                uint32_t v = w[x];
                if (in_block - lo < 32) v &= (1u << (in_block - lo)) - 1u;
                live += __popc(v);
            }
        }
    for (uint32_t off = 1; off < L; off <<= 1) live += __shfl_xor(live, off, 64);
    if (valid && sub == 0) {
        est[h] = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
        if (live_out) live_out[h] = live;
    }
}

static bool blocked_gather_ok(const Geo &G, uint32_t kprime, const uint32_t *hist)
{
    return G.blog >= 5 && kprime == G.k && hist == nullptr;
}

// ---------------------------------------------------------------------------
// k_estimate_learned: the gather of k_estimate (histogram path, window k)
// followed, in the same workgroup, by the learned estimator on the matrix
// cores.  Each wavefront's 64 hosts are fed to the network as four 16-row
// tiles built straight from the LDS histograms; the closed form is kept as
// the output where the network's result is not finite.
// ---------------------------------------------------------------------------
constexpr int kLearnMaxK = VATE_MLP_FEATURES - 3;

template <int W>
__global__ void __launch_bounds__(256) k_estimate_learned(Geo G, const uint8_t *__restrict__ pool,
                                                          const DevState *__restrict__ st,
                                                          const uint8_t *__restrict__ bitmap,
                                                          const uint32_t *__restrict__ hosts, uint32_t n,
                                                          const mlp::Packed *__restrict__ P,
                                                          float *__restrict__ est_out,
                                                          float *__restrict__ cf_out)
{
    constexpr int ROWS = (kLearnMaxK + 1) / 2 + 1;   // packed 16-bit bin pairs + live row
    __shared__ uint32_t hist_all[4][ROWS * 65];
    __shared__ __attribute__((aligned(16))) uint16_t xs_all[4][16 * mlp::LDS_STRIDE];
    __shared__ __attribute__((aligned(16))) uint16_t a1_all[4][16 * mlp::LDS_STRIDE];
    __shared__ float cf_all[4][64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t rows = (G.k + 1) / 2;
    uint32_t *my = hist_all[wave];
    for (uint32_t r = 0; r < rows; ++r) my[r * 65 + lane] = 0;
    const uint64_t active_pool = pool_active(st, G.k);
    const uint32_t bact0 = st->bact0;
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = h < n;
    const uint32_t key = host_key(G, valid ? hosts[h] : 0u);
    uint32_t live = 0;
    for (uint32_t i0 = 0; i0 < G.g; i0 += kEstU) {
        uint32_t pid[kEstU], byte[kEstU];
#pragma unroll
        for (int u = 0; u < kEstU; ++u) pid[u] = vat_pid(G, key, i0 + u);
#pragma unroll
        for (int u = 0; u < kEstU; ++u)
            byte[u] = (valid && i0 + u < G.g) ? bitmap[pid[u] >> 3] : 0u;
#pragma unroll
        for (int u = 0; u < kEstU; ++u) {
            if (!((byte[u] >> (pid[u] & 7u)) & 1u)) continue;
            const uint32_t val = load_at<W>(pool, pid[u], G.wb);
            const uint32_t d = value_dist(G, bact0, pid[u], val);
            ++live;
            atomicAdd(&my[(d >> 1) * 65 + lane], 1u << ((d & 1u) << 4));
        }
    }
    const float cf = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
    my[rows * 65 + lane] = live;
    cf_all[wave][lane] = cf;
    if (valid) cf_out[h] = cf;
    const float occupancy = (float)active_pool / (float)G.N;
    const float fg = (float)G.g;
    const int q = lane >> 4, c = lane & 15;
    uint16_t *xs = xs_all[wave];
    __syncthreads();
    const bool geo_off = mlp::env_geometry_off(P, G.k, G.g, G.c, G.wb);
    const mlp::EnvRange rng = mlp::env_range(P, (int)lane);   // this lane's feature in every row
    __shared__ uint32_t fell_wg;      // the workgroup's fallback hosts (one counter atomic per workgroup)
    if (threadIdx.x == 0) fell_wg = 0;
    uint32_t fell_wave = 0;
    for (int t = 0; t < 4; ++t) {
        // features of hosts 16t .. 16t+15 of this wavefront (row m = host - 16t);
        // lane f builds feature f of a row, so one ballot per row says whether
        // the host is outside the network's envelope
        uint32_t outside = geo_off ? 0xFFFFu : 0u;
        for (int e = lane; e < 16 * VATE_MLP_FEATURES; e += 64) {
            const int m = e >> 6, f = e & 63, host = 16 * t + m;
            float x = 0.f;
            if (f < (int)G.k)
                x = (float)((my[(f >> 1) * 65 + host] >> ((f & 1) << 4)) & 0xFFFFu) / fg;
            else if (f == (int)G.k)
                x = (float)my[rows * 65 + host] / fg;
            else if (f == (int)G.k + 1)
                x = occupancy;
            else if (f == (int)G.k + 2)
                x = logf(fmaxf(cf_all[wave][host], 1.0f)) * 0.0625f;
            const uint16_t xb = mlp::bf16_bits(x);
            xs[m * mlp::LDS_STRIDE + f] = xb;
            if (__ballot(mlp::env_outside(rng, xb))) outside |= 1u << m;
        }
        __syncthreads();
        float r4[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) r4[r] = logf(fmaxf(cf_all[wave][16 * t + 4 * q + r], 1.0f));
        mlp::f32x4 z1[4], z2[4];
        float a2v[4][4], o4[4];
        mlp::forward16(P, xs, a1_all[wave], r4, z1, z2, a2v, o4);
        bool fell = false;
        if (c < 4) {
            const int host = 16 * t + 4 * q + c;
            const uint32_t hg = blockIdx.x * blockDim.x + wave * 64 + host;
            if (hg < n) {
                const float e = expf(o4[c]);
                fell = ((outside >> (4 * q + c)) & 1u) || !isfinite(e);
                est_out[hg] = fell ? cf_all[wave][host] : e;
            }
        }
        fell_wave += (uint32_t)__popcll(__ballot(fell));
        __syncthreads();
    }
    if (lane == 0 && fell_wave) atomicAdd(&fell_wg, fell_wave);
    __syncthreads();
    if (threadIdx.x == 0) mlp::env_count(P, fell_wg);
}

#include "vate_part.h"

// ---------------------------------------------------------------------------
// Slice advance: BACT^0 = (BACT^0 + 1) mod 2k, t = t + 1 (Alg. 4 end of loop),
// census cleared for the new slice.
// ---------------------------------------------------------------------------
__global__ void k_advance(Geo G, DevState *__restrict__ st)
{
    if (threadIdx.x == 0) {
        st->bact0 = st->bact0 + 1 == G.twok ? 0 : st->bact0 + 1;
        st->t = st->t + 1;
    }
    for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) census_of(st)[d] = 0;
}

__global__ void k_set_clock(Geo G, DevState *__restrict__ st, unsigned long long t, uint32_t bact0)
{
    if (threadIdx.x == 0) {
        st->t = t;
        st->bact0 = bact0;
    }
    for (uint32_t d = threadIdx.x; d < G.k; d += blockDim.x) census_of(st)[d] = 0;
}

// ---------------------------------------------------------------------------
// k_preserve: PreserveAT (Alg. 3) over the two blocks whose ACT is now 0
// (block i0) or k (block i1), Cor. 1.  Block indices come from the device
// clock so a captured graph replays correctly.  Each 16-byte chunk that
// overlaps a due block is owned by exactly one thread (a chunk shared by both
// blocks belongs to the i0 pass), which rewrites it only if an AT changed.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void preserve_chunk(const Geo &G, uint4 *__restrict__ pool4, uint32_t bact0, uint64_t j,
                                               uint64_t max_chunks)
{
    constexpr uint64_t E = 128 / W;
    const uint32_t i0 = bact0 == 0 ? 0 : G.twok - bact0;                        // (BACT^0 + i0) mod 2k == 0
    const uint32_t i1 = bact0 <= G.k ? G.k - bact0 : G.twok + G.k - bact0;      // == k
    const uint64_t s0 = block_start(G, i0), e0 = block_start(G, i0 + 1);
    const uint64_t s1 = block_start(G, i1), e1 = block_start(G, i1 + 1);
    const uint64_t c0lo = s0 / E, c0hi = s0 < e0 ? (e0 + E - 1) / E : c0lo;
    const uint64_t c1lo = s1 / E, c1hi = s1 < e1 ? (e1 + E - 1) / E : c1lo;
    const bool second = j >= max_chunks;
    const uint64_t ch = second ? c1lo + (j - max_chunks) : c0lo + j;
    if (j >= 2 * max_chunks) return;
    if (ch >= (second ? c1hi : c0hi)) return;
    if (second && ch >= c0lo && ch < c0hi) return;
    uint4 v = pool4[ch];
    bool changed = false;
    for (uint32_t e = 0; e < E; ++e) {
        const uint64_t p = ch * E + e;
        const bool in0 = p >= s0 && p < e0, in1 = p >= s1 && p < e1;
        if (!in0 && !in1) continue;
        const uint32_t val = chunk_get<W>(v, e);
        bool mark;
        if (in0)   // ACT == 0: 0 <= Value <= k
            mark = val <= G.k;
        else       // ACT == k: k <= Value <= 2k-1, or Value == 0
            mark = (val >= G.k && val <= G.twok - 1) || val == 0;
        if (mark && val != G.twok) {
            chunk_set<W>(v, e, G.twok);
            changed = true;
        }
    }
    if (changed) pool4[ch] = v;
}

template <int W>
__global__ void __launch_bounds__(256) k_preserve(Geo G, uint4 *__restrict__ pool4,
                                                  const DevState *__restrict__ st, uint64_t max_chunks)
{
    preserve_chunk<W>(G, pool4, st->bact0, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, max_chunks);
}

// ---------------------------------------------------------------------------
// DR maintenance (the VDRE baseline of Sec. 5): at every slide each counter of
// the pool grows by one, saturating at k (Sec. 1).  The whole pool is read;
// a 16-byte chunk is written back only if one of its counters changed.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void dr_maintain_chunk(const Geo &G, uint4 *__restrict__ pool4, uint64_t ch)
{
    constexpr uint32_t E = 128 / W;
    uint4 v = pool4[ch];
    const uint32_t pat = replicate<W>(G.k);
    if (v.x == pat && v.y == pat && v.z == pat && v.w == pat) return;
    bool changed = false;
    for (uint32_t e = 0; e < E; ++e) {
        const uint32_t val = chunk_get<W>(v, e);
        if (val < G.k) {
            chunk_set<W>(v, e, val + 1);
            changed = true;
        }
    }
    if (changed) pool4[ch] = v;
}

template <int W>
__global__ void __launch_bounds__(256) k_dr_maintain(Geo G, uint4 *__restrict__ pool4, uint64_t nchunks)
{
    for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nchunks;
         ch += (uint64_t)gridDim.x * blockDim.x)
        dr_maintain_chunk<W>(G, pool4, ch);
}

#include "vate_batch_kernels.h"

}  // namespace vate

// ===========================================================================
// C ABI
// ===========================================================================
using namespace vate;

struct vate_sketch {
    vate_params p;
    Geo G;
    uint8_t *pool;
    DevState *st;
    uint8_t *bitmap;             // activity bitmap inside the state block
    unsigned long long *copies;  // k_census8's partial censuses inside the state block
    size_t pool_bytes, state_bytes;
    uint64_t max_block_chunks;   // chunks a due block can overlap
    int closed;                  // 1: slice ended, estimates allowed
    int dead;                    // sticky device error
    uint32_t lds_budget;         // dynamic LDS a partitioned-scatter workgroup may use (bytes)
    uint32_t n_cu;               // compute units of the device
    const void *plan_ws;         // workspace holding a host plan (vate_estimate_plan), or null
    uint64_t plan_n;             // its host count
    char err[256];
};

static int fail(vate_sketch *s, int code, const char *msg)
{
    if (s) {
        snprintf(s->err, sizeof(s->err), "%s", msg);
        if (code == VATE_E_DEVICE) s->dead = 1;
    }
    return code;
}

static int check_launch(vate_sketch *s, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[200];
        snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
        return fail(s, VATE_E_DEVICE, buf);
    }
    return VATE_OK;
}

static unsigned grid_for(uint64_t items, unsigned per_block, unsigned cap)
{
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (unsigned)std::min<uint64_t>(b, cap);
}

// Width dispatch: 4, 8 and 16 bits use their containers; any other width is
// the exact packing (template width 0).
template <class F>
static auto by_width(uint32_t w, F &&f)
{
    if (w == 4) return f(std::integral_constant<int, 4>{});
    if (w == 8) return f(std::integral_constant<int, 8>{});
    if (w == 16) return f(std::integral_constant<int, 16>{});
    return f(std::integral_constant<int, 0>{});
}

template <int W>
static void launch_init(vate_sketch *s, hipStream_t st)
{
    if constexpr (W == 0) {
        const uint64_t ng = s->G.N / 32;
        k_init_x<<<grid_for(ng, 256, 8192), 256, 0, st>>>(s->G, reinterpret_cast<uint32_t *>(s->pool), ng, s->st);
    } else {
        uint64_t nch = s->pool_bytes / 16;
        k_init<W><<<grid_for(nch, 256, 8192), 256, 0, st>>>(s->G, reinterpret_cast<uint4 *>(s->pool), nch, s->st,
                                                             s->copies);
    }
}

template <int W>
static void launch_census(vate_sketch *s, hipStream_t st)
{
    if constexpr (W == 0) {
        const uint64_t ng = s->G.N / 32;
        k_census_x<<<grid_for(ng, 256, 4096), 256, 0, st>>>(s->G, reinterpret_cast<const uint32_t *>(s->pool), ng,
                                                             s->st, s->bitmap);
    } else {
        uint64_t nch = s->pool_bytes / 16;
        if (W == 8 && s->G.k <= kCensus8Bins) {
            k_census8<<<grid_for(nch, 256 * kCensus8U, 4096), 256, 0, st>>>(
                s->G, reinterpret_cast<const uint4 *>(s->pool), nch, s->st, s->bitmap, s->copies);
            k_census_fold<<<1, 256, 0, st>>>(s->G, s->st, s->copies);
        } else {
            k_census<W><<<grid_for(nch, 256 * 4, 2048), 256, 0, st>>>(s->G, reinterpret_cast<const uint4 *>(s->pool),
                                                                       nch, s->st, s->bitmap);
        }
    }
}

template <int W>
static void launch_preserve(vate_sketch *s, hipStream_t st)
{
    uint64_t threads = 2 * s->max_block_chunks;
    if constexpr (W == 0)
        k_preserve_x<<<grid_for(threads, 256, 1u << 30), 256, 0, st>>>(s->G, reinterpret_cast<uint32_t *>(s->pool),
                                                                        s->st, s->max_block_chunks);
    else
        k_preserve<W><<<grid_for(threads, 256, 1u << 30), 256, 0, st>>>(s->G, reinterpret_cast<uint4 *>(s->pool),
                                                                         s->st, s->max_block_chunks);
}

template <int W>
static void launch_dr_maintain(vate_sketch *s, hipStream_t st)
{
    if constexpr (W == 0) {
        const uint64_t ng = s->G.N / 32;
        k_dr_maintain_x<<<grid_for(ng, 256, 8192), 256, 0, st>>>(s->G, reinterpret_cast<uint32_t *>(s->pool), ng);
    } else {
        const uint64_t nch = s->pool_bytes / 16;
        k_dr_maintain<W><<<grid_for(nch, 256, 8192), 256, 0, st>>>(s->G, reinterpret_cast<uint4 *>(s->pool), nch);
    }
}

template <int W>
static void launch_ingest(vate_sketch *s, const uint32_t *pairs, uint64_t n, hipStream_t st)
{
    unsigned blocks = grid_for(n, 1024, 1u << 30);
    if ((reinterpret_cast<uintptr_t>(pairs) & 15u) == 0)
        k_ingest<W, true><<<blocks, 256, 0, st>>>(s->G, pairs, n, s->pool, s->st);
    else
        k_ingest<W, false><<<blocks, 256, 0, st>>>(s->G, pairs, n, s->pool, s->st);
}

static void dispatch_init(vate_sketch *s, hipStream_t st)
{
    by_width(s->p.width, [&](auto W) { launch_init<decltype(W)::value>(s, st); });
}

static void dispatch_census(vate_sketch *s, hipStream_t st)
{
    by_width(s->p.width, [&](auto W) { launch_census<decltype(W)::value>(s, st); });
}

static int advance(vate_sketch *s, hipStream_t st)
{
    k_advance<<<1, 256, 0, st>>>(s->G, s->st);
    if (s->G.dr)
        by_width(s->p.width, [&](auto W) { launch_dr_maintain<decltype(W)::value>(s, st); });
    else
        by_width(s->p.width, [&](auto W) { launch_preserve<decltype(W)::value>(s, st); });
    s->closed = 0;
    return check_launch(s, "advance/preserve");
}

template <int W>
static void launch_estimate(vate_sketch *s, const uint32_t *hosts, uint32_t n, uint32_t kprime, float *est,
                            uint32_t *live, uint32_t *hist, hipStream_t st)
{
    if (blocked_gather_ok(s->G, kprime, hist)) {
        const uint32_t nb = (s->G.g + (1u << s->G.blog) - 1u) >> s->G.blog;
        uint32_t lg = 0;
        while ((1u << lg) < nb && lg < 6) ++lg;
        k_estimate_blocked<<<grid_for((uint64_t)n << lg, 256, 1u << 30), 256, 0, st>>>(
            s->G, s->st, reinterpret_cast<const uint32_t *>(s->bitmap), hosts, n, lg, est, live);
        return;
    }
    if (hist) {
        const uint32_t k = s->G.k;
        const unsigned threads = k <= 64 ? 256 : k <= 128 ? 128 : 64;
        const size_t lds = (size_t)(threads / 64) * ((k + 1) / 2 + 1) * 65 * sizeof(uint32_t);
        k_estimate<W, true><<<grid_for(n, threads, 1u << 30), threads, lds, st>>>(s->G, s->pool, s->st, s->bitmap,
                                                                                  hosts, n, kprime, est, live,
                                                                                  hist);
    } else {
        k_estimate<W, false><<<grid_for(n, 256, 1u << 30), 256, 0, st>>>(s->G, s->pool, s->st, s->bitmap,
                                                                         hosts, n, kprime, est, live, nullptr);
    }
}

template <int W>
static void launch_estimate_learned(vate_sketch *s, const uint32_t *hosts, uint32_t n, const void *weights,
                                    float *est, float *cf, hipStream_t st)
{
    k_estimate_learned<W><<<grid_for(n, 256, 1u << 30), 256, 0, st>>>(
        s->G, s->pool, s->st, s->bitmap, hosts, n, static_cast<const mlp::Packed *>(weights), est, cf);
}

// ---- partitioned estimate: geometry, workspace layout and launches ----
// part_geo returns false when the host count or g is outside the partitioned
// path's limits (g VATs of one host too many for one LDS sort) or the sketch
// uses the locality-blocked H; the entry points then use the direct gather.
static bool part_geo(const vate_sketch *s, uint64_t n, PartGeo *out)
{
    const Geo &G = s->G;
    if (G.blog > 0) return false;   // blocked VATs: the direct gather already reads whole blocks
    const uint32_t sl = G.c < kSliceLog2 ? G.c : kSliceLog2;
    const uint64_t ns = G.N >> sl;
    if (ns > kRunMaxSlices) return false;
    PartGeo p{};
    p.sl = sl;
    p.n_slices = (uint32_t)ns;
    p.bm_words = sl >= 5 ? 1u << (sl - 5) : 1u;
    p.xcd = ns >= 8 ? 1u : 0u;
    // Histogram rows of ceil((k+1)/2) words, made odd: an odd stride puts
    // the bins of different hosts in different LDS banks.
    p.rowp = ((G.k + 2u) / 2u) | 1u;
    // Hosts per subgroup: the largest count whose VATs' pids fit the scatter
    // threads' registers (kRunPerThread each), whose padded sort of 32-bit
    // entries (+ slice counters, keys) fits its LDS, and whose histograms fit
    // the finalize's LDS.
    const uint64_t nsp = (ns + 3) & ~3ull;
    auto lds_for = [&](uint64_t hosts) {   // counters, keys, 32-bit sort slots
        const uint64_t cap = (hosts * G.g + 3 * ns + 3) & ~3ull;
        return 4 * (nsp + ((hosts + 3) & ~3ull)) + 4 * cap;
    };
    uint64_t hosts = kRunMaxHosts;
    hosts = std::min<uint64_t>(hosts, (uint64_t)kRunPerThread * kRunThreads / G.g);
    hosts = std::min<uint64_t>(hosts, kFinHistBytes / (4ull * p.rowp));
    while (hosts > 0 && lds_for(hosts) > s->lds_budget) --hosts;
    if (hosts == 0) return false;
    p.hosts = (uint32_t)hosts;
    p.n_sub = (uint32_t)((n + hosts - 1) / hosts);
    p.vats = (uint32_t)hosts * G.g;
    p.cap = (uint32_t)((p.vats + 3ull * ns + 3) & ~3ull);
    p.region = (p.cap + 63u) & ~63u;
    // the lookup indexes the entries' 16-byte chunks with 32-bit integers
    if ((uint64_t)p.n_sub * (p.region / 4u) >= (1ull << 32)) return false;
    p.dq = kRunThreads / G.g;
    p.dr = kRunThreads % G.g;
    p.fast = G.a >= (1ull << sl) ? 1u : 0u;
    // Subgroups per finalize workgroup: the network takes hosts in tiles of
    // 64, so the count whose hosts leave the least of their last tile empty
    // (the fewest on a tie), as long as the histograms fit.
    {
        uint32_t best = 1;
        double waste = 1e30;
        for (uint32_t f = 1; f <= 16; ++f) {
            const uint64_t fh = f * hosts;
            if (fh * 4ull * p.rowp > kFinHistBytes) break;
            const double w = (double)(((fh + 63) / 64) * 64 - fh) / (double)fh;
            if (w < waste - 1e-9) waste = w, best = f;
        }
        p.fgroup = best;
    }
    p.lds_scatter = (uint32_t)lds_for(hosts);
    {   // lookup LDS: bits (whole 256-AT blocks + a sentinel word), rank tables,
        // run counters, then as many live ATs' distances as fit
        p.bm_words_lds = (p.bm_words + 1u + 7u) & ~7u;
        const uint32_t nblk = p.bm_words_lds / 8u, nsup = (nblk + 7u) / 8u;
        const uint32_t fixed = 4u * (p.bm_words_lds + nsup + (nblk + 1u) / 2u + kRunThreads);
        p.dist16 = G.k > 256 ? 1u : 0u;
        const uint32_t room = s->lds_budget > fixed ? s->lds_budget - fixed : 0u;
        p.dist_cap = room >> p.dist16;
        p.lds_lookup = (fixed + (p.dist_cap << p.dist16) + 15u) & ~15u;
        if (p.lds_lookup > s->lds_budget) p.lds_lookup = s->lds_budget & ~15u, p.dist_cap = (p.lds_lookup - fixed) >> p.dist16;
    }
    p.lds_final = p.fgroup * p.hosts * p.rowp * 4u + 4u;
    // Each slice's walk over the subgroups is cut into ranges, one workgroup
    // each, so that the launch has at least one workgroup per CU (each builds
    // its slice's LDS tables once); a range is a whole number of 64-subgroup
    // windows (one per wavefront at a time) and holds at least one window
    // per wavefront.
    const uint32_t per_round = kRunThreads;   // 16 wavefronts x 64 subgroups
    const uint32_t cus = std::max<uint32_t>(1u, s->n_cu);
    const uint32_t want = std::max<uint32_t>(1u, std::min<uint32_t>((cus + p.n_slices - 1u) / p.n_slices,
                                                                    p.n_sub / per_round));
    p.span = ((p.n_sub + want - 1u) / want + 63u) & ~63u;
    p.split = (p.n_sub + p.span - 1u) / p.span;
    *out = p;
    return true;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct RunWs {
    uint32_t *entries;          // [n_sub][region] sorted entries
    uint32_t *hits;             // [n_sub][region] live results (host << 16 | distance), packed at the front of each run's slots
    uint32_t *table;            // [n_sub][n_slices + 1] run starts and live counts
    uint32_t *heads;            // [n_sub][n_slices][4] each run's first four live results
    unsigned long long *cum;    // [k + 1] census prefix (several windows)
    size_t bytes;
};

static RunWs run_ws(const PartGeo &pg, uint32_t k, void *base)
{
    RunWs w;
    const uintptr_t p = reinterpret_cast<uintptr_t>(base);
    const size_t ents = (size_t)pg.n_sub * pg.region;
    size_t off = 0;
    w.entries = reinterpret_cast<uint32_t *>(p + off);
    off += align256(ents * 4);
    w.hits = reinterpret_cast<uint32_t *>(p + off);
    off += align256(ents * 4);
    w.table = reinterpret_cast<uint32_t *>(p + off);
    off += align256((size_t)pg.n_sub * (pg.n_slices + 1) * 4);
    w.heads = reinterpret_cast<uint32_t *>(p + off);
    off += align256((size_t)pg.n_sub * pg.n_slices * 16);
    w.cum = reinterpret_cast<unsigned long long *>(p + off);
    off += align256((size_t)(k + 1) * 8);
    w.bytes = off;
    return w;
}

static int set_lds_limit(vate_sketch *s, const void *fn, uint32_t bytes)
{
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return fail(s, VATE_E_DEVICE, hipGetErrorString(e));
    return VATE_OK;
}

// PART_ALL: scatter, lookup, finalize; PART_PLAN: the scatter only (the
// host plan); PART_RUN: lookup and finalize from an existing plan.
enum PartSteps { PART_ALL = 0, PART_PLAN = 1, PART_RUN = 2 };

template <int W, int MODE>
static int launch_part(vate_sketch *s, const PartGeo &pg, void *ws, const uint32_t *hosts, uint32_t n,
                       uint32_t kprime, float *est, uint32_t *live, uint32_t *hist, const Windows &win,
                       const void *weights, float *cf, hipStream_t st, int steps = PART_ALL)
{
    // The dynamic-LDS limits are a per-device function attribute: set once
    // per device (bit d of the mask) and instantiation.
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_set.load(std::memory_order_acquire) & bit)) {
        int rc = set_lds_limit(s, reinterpret_cast<const void *>(&k_run_scatter), s->lds_budget);
        if (rc == VATE_OK)
            rc = set_lds_limit(s, reinterpret_cast<const void *>(&k_run_lookup<W>), s->lds_budget);
        if (rc == VATE_OK)
            rc = set_lds_limit(s, reinterpret_cast<const void *>(&k_run_finalize<MODE>), kFinHistBytes + 16u);
        if (rc != VATE_OK) return rc;
        attr_set.fetch_or(bit, std::memory_order_release);
    }
    const RunWs w = run_ws(pg, s->p.k, ws);
    if (steps != PART_RUN)
        k_run_scatter<<<std::min(pg.n_sub, s->n_cu), kRunThreads, pg.lds_scatter, st>>>(s->G, pg, hosts, n, w.entries,
                                                                                       w.table);
    if (steps == PART_PLAN) return VATE_OK;
    k_run_lookup<W><<<pg.n_slices * pg.split, kRunThreads, pg.lds_lookup, st>>>(
        s->G, pg, s->pool, reinterpret_cast<const uint32_t *>(s->bitmap), s->st, w.entries, w.table, w.hits,
        w.heads);
    if (MODE == kFinMulti) k_census_prefix<<<1, 64, 0, st>>>(s->G, s->st, w.cum);
    k_run_finalize<MODE><<<(pg.n_sub + pg.fgroup - 1) / pg.fgroup, kFinThreads, pg.lds_final, st>>>(
        s->G, pg, s->st, n, kprime, w.hits, w.heads, w.table, est, live, hist, win, w.cum,
        static_cast<const mlp::Packed *>(weights), cf);
    return VATE_OK;
}

template <int MODE>
static int launch_part_w(vate_sketch *s, const PartGeo &pg, void *ws, const uint32_t *hosts, uint32_t n,
                         uint32_t kprime, float *est, uint32_t *live, uint32_t *hist, const Windows &win,
                         const void *weights, float *cf, hipStream_t st, int steps = PART_ALL)
{
    if (steps == PART_ALL && ws == s->plan_ws) s->plan_ws = nullptr;   // the plan is overwritten
    return by_width(s->p.width, [&](auto W) {
        return launch_part<decltype(W)::value, MODE>(s, pg, ws, hosts, n, kprime, est, live, hist, win, weights, cf,
                                                     st, steps);
    });
}

extern "C" {
int vate_estimate_learned_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes);

int vate_state_bytes(const vate_params *p, size_t *pool_bytes, size_t *state_bytes)
{
    Geo G;
    const char *why;
    int rc = make_geo(p, &G, &why);
    if (rc != VATE_OK) return rc;
    if (pool_bytes) *pool_bytes = (size_t)(G.N * p->width / 8);
    if (state_bytes) *state_bytes = state_bytes_for(p->k, G.N);
    return VATE_OK;
}

int vate_create(const vate_params *p, void *pool_dev, void *state_dev, void *stream, vate_sketch **out)
{
    if (!out) return VATE_E_INVAL;
    *out = nullptr;
    Geo G;
    const char *why;
    int rc = make_geo(p, &G, &why);
    if (rc != VATE_OK) return rc;
    if (!pool_dev || !state_dev) return VATE_E_INVAL;
    if ((reinterpret_cast<uintptr_t>(pool_dev) & 255u) || (reinterpret_cast<uintptr_t>(state_dev) & 255u))
        return VATE_E_INVAL;
    vate_sketch *s = new (std::nothrow) vate_sketch();
    if (!s) return VATE_E_NOMEM;
    s->p = *p;
    s->G = G;
    s->pool = static_cast<uint8_t *>(pool_dev);
    s->st = static_cast<DevState *>(state_dev);
    s->pool_bytes = (size_t)(G.N * p->width / 8);
    s->state_bytes = state_bytes_for(p->k, G.N);
    s->bitmap = static_cast<uint8_t *>(state_dev) + bitmap_offset(p->k);
    s->copies = reinterpret_cast<unsigned long long *>(static_cast<uint8_t *>(state_dev) + copies_offset(p->k, G.N));
    uint64_t maxb = 0;
    for (uint32_t i = 0; i < G.twok; ++i)
        maxb = std::max<uint64_t>(maxb, block_start(G, i + 1) - block_start(G, i));
    const bool exact = p->width != 4 && p->width != 8 && p->width != 16;
    const uint64_t E = exact ? 32 : 128 / p->width;      // counters per word group / 16-byte chunk
    s->max_block_chunks = (maxb + E - 1) / E + 1;
    {   // LDS a workgroup may use: the largest the device reports (gfx950: 160 KiB)
        int dev = 0, lds = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess)
            for (hipDeviceAttribute_t a : {hipDeviceAttributeMaxSharedMemoryPerBlock,
                                           hipDeviceAttributeSharedMemPerBlockOptin,
                                           hipDeviceAttributeMaxSharedMemoryPerMultiprocessor}) {
                int v = 0;
                if (hipDeviceGetAttribute(&v, a, dev) == hipSuccess && v > lds) lds = v;
            }
        s->lds_budget = std::min<uint32_t>((uint32_t)lds, kRunLdsMax) - kRunLdsStatic;
        int cus = 0;
        s->n_cu = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0
                      ? (uint32_t)cus
                      : 256u;
    }
    s->closed = 0;
    s->dead = 0;
    s->err[0] = 0;
    dispatch_init(s, static_cast<hipStream_t>(stream));
    rc = check_launch(s, "init");
    if (rc != VATE_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return VATE_OK;
}

int vate_ingest(vate_sketch *s, const uint32_t *pairs_dev, size_t n, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (n > 0 && (!pairs_dev || (reinterpret_cast<uintptr_t>(pairs_dev) & 7u)))
        return fail(s, VATE_E_INVAL, "pairs must be non-NULL and 8-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->closed) {
        int rc = advance(s, st);
        if (rc != VATE_OK) return rc;
    }
    if (n == 0) return VATE_OK;
    by_width(s->p.width, [&](auto W) { launch_ingest<decltype(W)::value>(s, pairs_dev, n, st); });
    return check_launch(s, "ingest");
}

int vate_close_slice(vate_sketch *s, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->closed) {
        int rc = advance(s, st);
        if (rc != VATE_OK) return rc;
    }
    dispatch_census(s, st);
    int rc = check_launch(s, "census");
    if (rc != VATE_OK) return rc;
    s->closed = 1;
    return VATE_OK;
}

int vate_estimate(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, uint32_t kprime, float *est_dev,
                  uint32_t *live_dev, uint32_t *hist_dev, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (kprime < 1 || kprime > s->p.k) return fail(s, VATE_E_INVAL, "k' must be in [1, k]");
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    if (hist_dev && s->p.k > (uint32_t)kMaxHistK)
        return fail(s, VATE_E_UNSUPPORTED, "per-host histogram needs k <= 256");
    if (n_hosts == 0) return VATE_OK;
    if (!hosts_dev || !est_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(live_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(hist_dev) & 3u))
        return fail(s, VATE_E_INVAL, "hosts/est/live/hist must be non-NULL (live, hist may be NULL) and 4-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t n = (uint32_t)n_hosts;
    by_width(s->p.width, [&](auto W) {
        launch_estimate<decltype(W)::value>(s, hosts_dev, n, kprime, est_dev, live_dev, hist_dev, st);
    });
    return check_launch(s, "estimate");
}

int vate_estimate_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes)
{
    if (!s || !bytes) return VATE_E_INVAL;
    if (n_hosts > 0xFFFFFFFFull - 1024) return VATE_E_INVAL;
    PartGeo pg;
    *bytes = part_geo(s, n_hosts, &pg) ? run_ws(pg, s->p.k, nullptr).bytes : 256;
    return VATE_OK;
}

}  // extern "C"

// vate_estimate_ws and vate_estimate_noalloc: the same checks and launches;
// `what` names the entry point in error messages.
static int estimate_ws_impl(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, uint32_t kprime,
                            float *est_dev, uint32_t *live_dev, uint32_t *hist_dev, void *workspace_dev,
                            size_t workspace_bytes, hipStream_t st, const char *what)
{
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (kprime < 1 || kprime > s->p.k) return fail(s, VATE_E_INVAL, "k' must be in [1, k]");
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    if (n_hosts == 0) return VATE_OK;
    size_t need = 0;
    vate_estimate_workspace_bytes(s, n_hosts, &need);
    if (!workspace_dev || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace_dev) & 255u))
        return fail(s, VATE_E_INVAL, "workspace missing, too small or not 256-byte aligned");
    if (!hosts_dev || !est_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(live_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(hist_dev) & 3u))
        return fail(s, VATE_E_INVAL, "hosts/est/live/hist must be non-NULL (live, hist may be NULL) and 4-byte aligned");
    const uint32_t n = (uint32_t)n_hosts;
    PartGeo pg;
    if (!part_geo(s, n, &pg)) {      // outside the partitioned limits: direct gather
        if (hist_dev && s->p.k > (uint32_t)kMaxHistK)
            return fail(s, VATE_E_UNSUPPORTED, "per-host histogram of this geometry needs k <= 256");
        by_width(s->p.width, [&](auto W) {
            launch_estimate<decltype(W)::value>(s, hosts_dev, n, kprime, est_dev, live_dev, hist_dev, st);
        });
        return check_launch(s, what);
    }
    const int rc = launch_part_w<kFinClosedForm>(s, pg, workspace_dev, hosts_dev, n, kprime, est_dev, live_dev,
                                                 hist_dev, Windows{}, nullptr, nullptr, st);
    if (rc != VATE_OK) return rc;
    return check_launch(s, what);
}

// Workspace of vate_estimate_noalloc: a fixed array in device memory.  Each
// GPU the library runs on holds its own copy from module load until the
// process ends.  Host code never uses the array's name as a device address
// (on the host it names a stand-in): the address is looked up once per
// device with hipGetSymbolAddress, and that pointer is what the launches get.
static __device__ __align__(256) uint8_t scratch[VATE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::atomic<void *> g_scratch_dev[kMaxDevices];

// Device address of the current device's scratch array (looked up on the
// first call per device), or null with the HIP error in *err.
static void *scratch_address(hipError_t *err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    void *p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (p) return p;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_dev[dev].store(p, std::memory_order_release);
    return p;
}

extern "C" {
int vate_estimate_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, uint32_t kprime, float *est_dev,
                     uint32_t *live_dev, uint32_t *hist_dev, void *workspace_dev, size_t workspace_bytes,
                     void *stream)
{
    if (!s) return VATE_E_INVAL;
    return estimate_ws_impl(s, hosts_dev, n_hosts, kprime, est_dev, live_dev, hist_dev, workspace_dev,
                            workspace_bytes, static_cast<hipStream_t>(stream), "estimate_ws");
}

int vate_estimate_noalloc(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, uint32_t kprime,
                          float *est_dev, uint32_t *live_dev, uint32_t *hist_dev, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    size_t need = 0;
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    vate_estimate_workspace_bytes(s, n_hosts, &need);
    if (need > VATE_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof(buf), "estimate_noalloc: %zu hosts need %zu bytes of workspace, more than the %u of the "
                 "fixed scratch (use vate_estimate_ws)", n_hosts, need, (unsigned)VATE_NOALLOC_SCRATCH_BYTES);
        return fail(s, VATE_E_INVAL, buf);
    }
    hipError_t e = hipSuccess;
    void *ws = scratch_address(&e);
    if (!ws) return fail(s, VATE_E_DEVICE, hipGetErrorString(e));
    return estimate_ws_impl(s, hosts_dev, n_hosts, kprime, est_dev, live_dev, hist_dev, ws,
                            VATE_NOALLOC_SCRATCH_BYTES, static_cast<hipStream_t>(stream), "estimate_noalloc");
}

int vate_estimate_plan(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, void *workspace_dev,
                       size_t workspace_bytes, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (n_hosts == 0 || n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "need 1 .. 2^32-1025 hosts");
    PartGeo pg;
    if (!part_geo(s, n_hosts, &pg))
        return fail(s, VATE_E_UNSUPPORTED, "no partitioned plan for this sketch (use vate_estimate)");
    size_t need = 0;
    vate_estimate_workspace_bytes(s, n_hosts, &need);
    if (!workspace_dev || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace_dev) & 255u))
        return fail(s, VATE_E_INVAL, "workspace missing, too small or not 256-byte aligned");
    if (!hosts_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u))
        return fail(s, VATE_E_INVAL, "hosts must be non-NULL and 4-byte aligned");
    const int rc = launch_part_w<kFinClosedForm>(s, pg, workspace_dev, hosts_dev, (uint32_t)n_hosts, s->p.k, nullptr,
                                                 nullptr, nullptr, Windows{}, nullptr, nullptr,
                                                 static_cast<hipStream_t>(stream), PART_PLAN);
    if (rc != VATE_OK) return rc;
    s->plan_ws = workspace_dev;
    s->plan_n = n_hosts;
    return check_launch(s, "estimate_plan");
}

// A run needs a closed slice and the plan made for this workspace and host count.
static int check_plan(vate_sketch *s, size_t n_hosts, const void *workspace_dev, size_t workspace_bytes, size_t need,
                      PartGeo *pg)
{
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (!workspace_dev || workspace_dev != s->plan_ws || n_hosts != s->plan_n)
        return fail(s, VATE_E_STATE, "no plan for this workspace and host count (call vate_estimate_plan)");
    if (workspace_bytes < need) return fail(s, VATE_E_INVAL, "workspace too small");
    if (!part_geo(s, n_hosts, pg)) return fail(s, VATE_E_STATE, "plan geometry unavailable");
    return VATE_OK;
}

int vate_estimate_run(vate_sketch *s, size_t n_hosts, uint32_t kprime, float *est_dev, uint32_t *live_dev,
                      uint32_t *hist_dev, void *workspace_dev, size_t workspace_bytes, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (kprime < 1 || kprime > s->p.k) return fail(s, VATE_E_INVAL, "k' must be in [1, k]");
    size_t need = 0;
    vate_estimate_workspace_bytes(s, n_hosts, &need);
    PartGeo pg;
    int rc = check_plan(s, n_hosts, workspace_dev, workspace_bytes, need, &pg);
    if (rc != VATE_OK) return rc;
    if (!est_dev || (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(live_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(hist_dev) & 3u))
        return fail(s, VATE_E_INVAL, "est/live/hist must be 4-byte aligned, est non-NULL");
    rc = launch_part_w<kFinClosedForm>(s, pg, workspace_dev, nullptr, (uint32_t)n_hosts, kprime, est_dev, live_dev,
                                       hist_dev, Windows{}, nullptr, nullptr, static_cast<hipStream_t>(stream),
                                       PART_RUN);
    if (rc != VATE_OK) return rc;
    return check_launch(s, "estimate_run");
}

int vate_estimate_learned_run(vate_sketch *s, size_t n_hosts, const void *weights_dev, float *est_dev,
                              float *est_cf_dev, void *workspace_dev, size_t workspace_bytes, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->p.k > (uint32_t)kLearnMaxK) return fail(s, VATE_E_UNSUPPORTED, "learned estimator needs k + 3 <= 64");
    size_t need = 0;
    vate_estimate_learned_workspace_bytes(s, n_hosts, &need);
    PartGeo pg;
    int rc = check_plan(s, n_hosts, workspace_dev, workspace_bytes, need, &pg);
    if (rc != VATE_OK) return rc;
    if (!est_dev || !est_cf_dev || !weights_dev || (reinterpret_cast<uintptr_t>(est_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_cf_dev) & 3u) || (reinterpret_cast<uintptr_t>(weights_dev) & 255u))
        return fail(s, VATE_E_INVAL, "est/est_cf must be 4-byte and weights 256-byte aligned, non-NULL");
    rc = launch_part_w<kFinLearned>(s, pg, workspace_dev, nullptr, (uint32_t)n_hosts, s->p.k, est_dev, nullptr,
                                    nullptr, Windows{}, weights_dev, est_cf_dev, static_cast<hipStream_t>(stream),
                                    PART_RUN);
    if (rc != VATE_OK) return rc;
    return check_launch(s, "estimate_learned_run");
}

int vate_estimate_learned_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, const void *weights_dev,
                             float *est_dev, float *est_cf_dev, void *workspace_dev, size_t workspace_bytes,
                             void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (s->p.k > (uint32_t)kLearnMaxK) return fail(s, VATE_E_UNSUPPORTED, "learned estimator needs k + 3 <= 64");
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    if (n_hosts == 0) return VATE_OK;
    size_t need = 0;
    vate_estimate_learned_workspace_bytes(s, n_hosts, &need);
    if (!workspace_dev || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace_dev) & 255u))
        return fail(s, VATE_E_INVAL, "workspace missing, too small or not 256-byte aligned");
    if (!hosts_dev || !est_dev || !est_cf_dev || !weights_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(est_cf_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(weights_dev) & 255u))
        return fail(s, VATE_E_INVAL, "hosts/est/est_cf must be 4-byte and weights 256-byte aligned, non-NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t n = (uint32_t)n_hosts;
    PartGeo pg;
    if (!part_geo(s, n, &pg)) {      // outside the partitioned limits: fused direct gather
        by_width(s->p.width, [&](auto W) {
            launch_estimate_learned<decltype(W)::value>(s, hosts_dev, n, weights_dev, est_dev, est_cf_dev, st);
        });
        return check_launch(s, "estimate_learned_ws");
    }
    const int rc = launch_part_w<kFinLearned>(s, pg, workspace_dev, hosts_dev, n, s->p.k, est_dev, nullptr, nullptr,
                                              Windows{}, weights_dev, est_cf_dev, st);
    if (rc != VATE_OK) return rc;
    return check_launch(s, "estimate_learned_ws");
}

int vate_estimate_multi_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes)
{
    if (!s || !bytes) return VATE_E_INVAL;
    if (n_hosts > 0xFFFFFFFFull - 1024) return VATE_E_INVAL;
    PartGeo pg;
    if (part_geo(s, n_hosts, &pg))
        *bytes = run_ws(pg, s->p.k, nullptr).bytes;
    else    // direct gather into full histograms, then the windows
        *bytes = align256((size_t)n_hosts * (s->p.k + 1) * 4) + align256(8ull * (s->p.k + 1));
    return VATE_OK;
}

int vate_estimate_multi_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, const uint32_t *kprimes,
                           uint32_t m, float *est_dev, void *workspace_dev, size_t workspace_bytes, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (!kprimes || m < 1 || m > kMaxWindows) return fail(s, VATE_E_INVAL, "need 1..64 windows");
    Windows win;
    win.m = m;
    for (uint32_t j = 0; j < m; ++j) {
        if (kprimes[j] < 1 || kprimes[j] > s->p.k || (j > 0 && kprimes[j] <= kprimes[j - 1]))
            return fail(s, VATE_E_INVAL, "windows must be ascending, distinct and in [1, k]");
        win.kp[j] = kprimes[j];
    }
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    if (n_hosts == 0) return VATE_OK;
    size_t need = 0;
    vate_estimate_multi_workspace_bytes(s, n_hosts, &need);
    if (!workspace_dev || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace_dev) & 255u))
        return fail(s, VATE_E_INVAL, "workspace missing, too small or not 256-byte aligned");
    if (!hosts_dev || !est_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u))
        return fail(s, VATE_E_INVAL, "hosts/est must be non-NULL and 4-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t n = (uint32_t)n_hosts;
    PartGeo pg;
    if (part_geo(s, n, &pg)) {
        const int rc = launch_part_w<kFinMulti>(s, pg, workspace_dev, hosts_dev, n, s->p.k, est_dev, nullptr,
                                                nullptr, win, nullptr, nullptr, st);
        if (rc != VATE_OK) return rc;
        return check_launch(s, "estimate_multi_ws");
    }
    if (s->p.k > (uint32_t)kMaxHistK)
        return fail(s, VATE_E_UNSUPPORTED, "several windows for this geometry need k <= 256");
    uint8_t *ws = static_cast<uint8_t *>(workspace_dev);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws);
    unsigned long long *cum = reinterpret_cast<unsigned long long *>(ws + align256((size_t)n * (s->p.k + 1) * 4));
    // the direct gather for window k fills the per-host histograms (est is scratch here)
    by_width(s->p.width, [&](auto W) {
        launch_estimate<decltype(W)::value>(s, hosts_dev, n, s->p.k, est_dev, nullptr, hist, st);
    });
    k_census_prefix<<<1, 64, 0, st>>>(s->G, s->st, cum);
    k_multi_from_hist<<<grid_for(n, 256, 1u << 30), 256, 0, st>>>(s->G, n, win, cum, hist, est_dev);
    return check_launch(s, "estimate_multi_ws");
}

int vate_estimate_learned_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes)
{
    if (!s || !bytes) return VATE_E_INVAL;
    if (n_hosts > 0xFFFFFFFFull - 1024) return VATE_E_INVAL;
    PartGeo pg;
    *bytes = part_geo(s, n_hosts, &pg) ? run_ws(pg, s->p.k, nullptr).bytes : 256;
    return VATE_OK;
}

int vate_estimate_learned(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts, const void *weights_dev,
                          float *est_dev, float *est_cf_dev, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "estimate needs a closed slice (call vate_close_slice)");
    if (s->p.k > (uint32_t)kLearnMaxK) return fail(s, VATE_E_UNSUPPORTED, "learned estimator needs k + 3 <= 64");
    if (n_hosts > 0xFFFFFFFFull - 1024) return fail(s, VATE_E_INVAL, "too many hosts");
    if (n_hosts == 0) return VATE_OK;
    if (!hosts_dev || !est_dev || !est_cf_dev || !weights_dev || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(est_cf_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(weights_dev) & 255u))
        return fail(s, VATE_E_INVAL, "hosts/est/est_cf must be 4-byte and weights 256-byte aligned, non-NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t n = (uint32_t)n_hosts;
    by_width(s->p.width, [&](auto W) {
        launch_estimate_learned<decltype(W)::value>(s, hosts_dev, n, weights_dev, est_dev, est_cf_dev, st);
    });
    return check_launch(s, "estimate_learned");
}

int vate_read_census(vate_sketch *s, uint64_t *census_host, void *stream)
{
    if (!s || !census_host) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (!s->closed) return fail(s, VATE_E_STATE, "census needs a closed slice");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(census_host, census_of(s->st), 8ull * s->p.k, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(s, VATE_E_DEVICE, hipGetErrorString(e));
    uint64_t act = 0;
    for (uint32_t d = 0; d < s->p.k; ++d) act += census_host[d];
    census_host[s->p.k] = s->G.N - act;
    return VATE_OK;
}

int vate_read_state(vate_sketch *s, void *pool_dst, uint64_t *t, uint32_t *bact0, int *closed, void *stream)
{
    if (!s) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);
    DevState hdr;
    if (e == hipSuccess && pool_dst) e = hipMemcpy(pool_dst, s->pool, s->pool_bytes, hipMemcpyDefault);
    if (e == hipSuccess) e = hipMemcpy(&hdr, s->st, kStateHeader, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(s, VATE_E_DEVICE, hipGetErrorString(e));
    if (t) *t = hdr.t;
    if (bact0) *bact0 = hdr.bact0;
    if (closed) *closed = s->closed;
    return VATE_OK;
}

int vate_load_state(vate_sketch *s, const void *pool_src, uint64_t t, uint32_t bact0, int closed, void *stream)
{
    if (!s || !pool_src) return VATE_E_INVAL;
    if (s->dead) return VATE_E_DEVICE;
    if (bact0 >= s->G.twok) return fail(s, VATE_E_INVAL, "bact0 must be < 2k");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(s->pool, pool_src, s->pool_bytes, hipMemcpyDefault, st);
    if (e != hipSuccess) return fail(s, VATE_E_DEVICE, hipGetErrorString(e));
    k_set_clock<<<1, 256, 0, st>>>(s->G, s->st, (unsigned long long)t, bact0);
    int rc = check_launch(s, "load_state");
    if (rc != VATE_OK) return rc;
    s->closed = 0;
    if (closed) {
        dispatch_census(s, st);
        rc = check_launch(s, "census");
        if (rc != VATE_OK) return rc;
        s->closed = 1;
    }
    return VATE_OK;
}

const char *vate_last_error(const vate_sketch *s)
{
    return s ? s->err : "";
}

const char *vate_status_string(int code)
{
    switch (code) {
    case VATE_OK: return "ok";
    case VATE_E_INVAL: return "invalid argument";
    case VATE_E_STATE: return "call not allowed in the current slice phase";
    case VATE_E_DEVICE: return "HIP device error";
    case VATE_E_NOMEM: return "out of host memory";
    case VATE_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

void vate_destroy(vate_sketch *s)
{
    delete s;
}

uint32_t vate_host_hash(const vate_params *p, uint32_t which, uint32_t x, uint32_t i)
{
    Geo G;
    const char *why;
    if (make_geo(p, &G, &why) != VATE_OK) return 0xFFFFFFFFu;
    if (which == 0) return bh(G, x);
    if (which == 1) return vat_pid(G, host_key(G, x), i);
    return 0xFFFFFFFFu;
}

uint32_t vate_host_block(const vate_params *p, uint64_t pid)
{
    Geo G;
    const char *why;
    if (make_geo(p, &G, &why) != VATE_OK || pid >= G.N) return 0xFFFFFFFFu;
    return block_of(G, (uint32_t)pid);
}

}  // extern "C"

#include "vate_batch_api.h"
