// Partitioned estimate: the g CheckAT lookups of every host (Alg. 4's
// estimate loop, Alg. 1) routed to the pool slice that holds their AT,
// resolved out of LDS, and routed back.  Included into vate.hip inside
// namespace vate.
//
// The direct gather reads one random cache line per VAT anywhere in the
// pool, so it is bound by line fills from beyond L2.  Here the pool is cut
// into slices of 2^20 ATs, whose activity bits (the census bitmap: CheckAT
// for the window k) fill 128 KiB of LDS:
//
//  k_run_scatter  persistent workgroups, one subgroup of hosts at a time.
//                 Hashes the subgroup's VATs once (each pid stays in a
//                 register, 40 per thread), counts them per slice in LDS and
//                 places 32-bit entries (host within subgroup, AT within
//                 slice) by an LDS counting sort, then copies them to the
//                 workspace as one coalesced stream.  Every (subgroup, slice)
//                 run starts on a 4-entry boundary (padded with the slice's
//                 sentinel entry), so no 16-byte chunk is shared by two runs.
//                 Run starts, in chunks, go to the subgroup's row of the run
//                 table.
//  k_run_lookup   one slice's bits in LDS per workgroup (a slice's walk over
//                 the subgroups may be split over a few workgroups; the
//                 slices of one XCD are contiguous).  Where they fit, the
//                 distances (Eq. 5) of the slice's live ATs are computed once
//                 into LDS in slice order, indexed by the AT's rank among the
//                 live bits.  A wavefront takes the runs of 64 subgroups as one
//                 flat list of chunks and tests every entry's bit; only the
//                 live ones (active for window k: about 1 % of the VATs in the
//                 40 Gb/s steady state) take a slot of their run from an LDS
//                 counter and write (host within subgroup, distance): the
//                 run's first four into its 16-byte cell of a dense
//                 [subgroup][slice] array, any more into the entries' own
//                 positions of the result array.  The run's live count goes
//                 beside its start in the table.
//  k_run_finalize a few subgroups per workgroup.  Reads the live results of
//                 their runs (a subgroup's cells are contiguous, so mostly
//                 whole lines), builds each host's distance histogram in LDS
//                 (the inactive bin k, g minus the rest, only for the
//                 histogram output) and forms Eq. 11 for
//                 k', several windows, or the learned estimate (the network
//                 fed from the LDS histograms, 16 hosts per wavefront).
//
// HBM traffic per VAT: the 4-byte entry written and read back once; per live
// VAT 4 bytes of result written and read back (in 16-byte run cells).

constexpr uint32_t kRunThreads = 1024;                          // scatter / lookup workgroup
constexpr uint32_t kRunPerThread = 40;                          // VATs hashed per scatter thread (pids held in registers)
constexpr uint32_t kRunLdsMax = 160u * 1024u;                   // gfx950 LDS per workgroup
constexpr uint32_t kRunLdsStatic = 64u;                         // k_run_scatter's static LDS (wsum)
constexpr uint32_t kSliceLog2 = 20;                             // ATs per slice: 2^20, 128 KiB of activity bits
constexpr uint32_t kRunMaxSlices = 4096;                        // any pool up to 2^32 ATs
constexpr uint32_t kRunMaxHosts = 1024;                         // hosts per subgroup
constexpr uint32_t kFinThreads = 256;
constexpr uint32_t kLookU = 8;                                  // 16-byte entry chunks per lane and lookup pass
constexpr uint32_t kFinHistBytes = 64u * 1024u;                 // per-subgroup histogram ceiling

struct PartGeo {
    uint32_t sl;          // ATs per slice = 2^sl
    uint32_t n_slices;    // N >> sl
    uint32_t bm_words;    // 32-bit bitmap words per slice (at least one)
    uint32_t bm_words_lds;// the lookup's LDS words for them: whole 256-AT blocks and a zero sentinel word after
    uint32_t dist_cap;    // live ATs of a slice whose distances the lookup keeps in LDS
    uint32_t dist16;      // distances take 16 bits (k > 256)
    uint32_t hosts;       // hosts per subgroup
    uint32_t n_sub;       // subgroups
    uint32_t vats;        // hosts * g
    uint32_t cap;         // padded entries per subgroup at most: vats + 3 n_slices, rounded up to 4
    uint32_t region;      // entries between subgroup regions (cap rounded up to 64)
    uint32_t dq, dr;      // kRunThreads = dq * g + dr
    uint32_t fast;        // every block holds >= 2^sl ATs: a slice meets at most two blocks
    uint32_t rowp;        // u32 words per packed 16-bit histogram row: ceil((k + 1) / 2), made odd
    uint32_t xcd;         // give the workgroups of one slice to one XCD
    uint32_t split;       // lookup workgroups per slice, each over a range of subgroups
    uint32_t span;        // subgroups per range (a multiple of kGroupRuns)
    uint32_t fgroup;      // subgroups per finalize workgroup
    uint32_t lds_scatter, lds_lookup, lds_final;
};

// Run table: row s (n_slices + 1 cells of 32 bits) belongs to subgroup s.
// Cell b < n_slices: the start of run (s, b) in 4-entry chunks (low half,
// written by the scatter) and its live count (high half, written by the
// lookup); cell n_slices: the subgroup's padded length in chunks.

// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pad4(uint32_t x) { return (x + 3u) & ~3u; }

__global__ void __launch_bounds__(kRunThreads) k_run_scatter(Geo G, PartGeo PG, const uint32_t *__restrict__ hosts,
                                                            uint32_t n, uint32_t *__restrict__ entries,
                                                            uint32_t *__restrict__ table)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ uint32_t wsum[kRunThreads / 64];
    const uint32_t nsp = (PG.n_slices + 3u) & ~3u;
    const uint32_t nkp = (PG.hosts + 3u) & ~3u;
    uint32_t *cnt = lds;                  // per-slice counts, then cursors
    uint32_t *keys = lds + nsp;           // host keys
    uint32_t *sorted = keys + nkp;        // entries by slice, runs padded to 4 (16-byte aligned)
    const uint32_t t = threadIdx.x;
    const uint32_t sl = PG.sl, mask = (1u << sl) - 1u;
    const uint32_t host_t0 = t / G.g, i_t0 = t - host_t0 * G.g;
    const uint32_t d_ik = PG.dr * kPhi, g_ik = G.g * kPhi;

    // Workgroups persist: workgroup x sorts subgroups x, x + grid, ...  The
    // host ids of its next subgroup are loaded (one per thread: hosts per
    // subgroup <= workgroup size) while the current one is sorted.
    uint32_t s = blockIdx.x;
    for (uint32_t q = t; q < nsp; q += kRunThreads) cnt[q] = 0;
    if (s < PG.n_sub) {
        const uint32_t h0 = s * PG.hosts, nh = min(PG.hosts, n - h0);
        if (t < nh) keys[t] = host_key(G, hosts[h0 + t]);
    }
    __syncthreads();
    for (; s < PG.n_sub; s += gridDim.x) {
        const uint32_t h0 = s * PG.hosts;
        const uint32_t nh = min(PG.hosts, n - h0);
        const uint32_t nv = nh * G.g;
        const uint32_t sn = s + gridDim.x;
        const uint32_t nh_next = sn < PG.n_sub ? min(PG.hosts, n - sn * PG.hosts) : 0u;
        uint32_t aip_next = 0;
        if (t < nh_next) aip_next = hosts[(size_t)sn * PG.hosts + t];
        // Opaque per iteration, so the compiler does not hoist the VATs' LDS
        // addresses out of the loop (they would not fit in registers).
        uint32_t host_t = host_t0, i_t = i_t0;
        asm volatile("" : "+v"(host_t), "+v"(i_t));

        // VAT v = t + j * kRunThreads (v < nv) of the subgroup is VAT
        // i = v mod g of host v / g.  H's multiplier i * phi is carried along
        // (mod 2^32); when g divides the workgroup size, i (and i * phi) stay
        // fixed and only the host advances.  H(aip, i) = top c bits of the
        // mix (shift = 32 - c is at most 31).  Each VAT's pid stays in a
        // register until it is placed.
        uint32_t pid[kRunPerThread];
        // When g is a multiple of 64 (and divides the workgroup size), the 64
        // lanes of a wavefront hash VATs of one host in every round: its key
        // is one broadcast LDS read and the round's bound a scalar test.  All
        // hashes come first (the key reads then wait for no LDS atomic), then
        // the counts.  Keys past the subgroup's hosts (the LDS after the keys
        // holds the sort slots) give pids that are never counted or placed.
        const bool wave_host = PG.dr == 0 && (G.g & 63u) == 0;
        const uint32_t host_w = __builtin_amdgcn_readfirstlane(host_t);
        if (wave_host) {
            const uint32_t ik = i_t * kPhi;
            const uint32_t *kw = keys + host_w;
            if (PG.dq == 1) {
#pragma unroll
                for (uint32_t j = 0; j < kRunPerThread; ++j) pid[j] = mix(kw[j] ^ ik) >> G.shift;
            } else {
#pragma unroll
                for (uint32_t j = 0; j < kRunPerThread; ++j) pid[j] = mix(kw[j * PG.dq] ^ ik) >> G.shift;
            }
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j)
                if (host_w + j * PG.dq < nh) atomicAdd(&cnt[pid[j] >> sl], 1u);
        } else if (PG.dr == 0) {
            const uint32_t ik = i_t * kPhi;
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                const uint32_t host = host_t + j * PG.dq;
                pid[j] = 0;
                if (t + j * kRunThreads < nv) {
                    pid[j] = mix(keys[host] ^ ik) >> G.shift;
                    atomicAdd(&cnt[pid[j] >> sl], 1u);
                }
            }
        } else {
            uint32_t host = host_t, i = i_t, ik = i_t * kPhi;
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                pid[j] = 0;
                if (t + j * kRunThreads < nv) {
                    pid[j] = mix(keys[host] ^ ik) >> G.shift;
                    atomicAdd(&cnt[pid[j] >> sl], 1u);
                }
                const bool wrap = i + PG.dr >= G.g;
                i = i + PG.dr - (wrap ? G.g : 0u);
                ik = ik + d_ik - (wrap ? g_ik : 0u);
                host += PG.dq + (wrap ? 1u : 0u);
            }
        }
        __syncthreads();
        // The keys are not read again in this subgroup: the next one's take
        // their place now, while no store of this workgroup is in flight (a
        // wait for the host id load after the copy-out below would also wait
        // for every store of the copy-out).
        if (t < nh_next) keys[t] = host_key(G, aip_next);

        // Exclusive scan of the padded slice counts; thread t owns slices
        // [t ps, (t+1) ps).  Run starts become the cursors, padding slots
        // are marked.
        const uint32_t ps = (PG.n_slices + kRunThreads - 1) / kRunThreads;
        const uint32_t b0 = t * ps;
        uint32_t mine = 0;
        for (uint32_t q = 0; q < ps; ++q)
            if (b0 + q < PG.n_slices) mine += pad4(cnt[b0 + q]);
        const uint32_t lane = t & 63u, wv = t >> 6;
        uint32_t incl = mine;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= (uint32_t)off) incl += y;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint32_t run = incl - mine;
        for (uint32_t q = 0; q < wv; ++q) run += wsum[q];
        for (uint32_t q = 0; q < ps; ++q) {
            const uint32_t b = b0 + q;
            if (b >= PG.n_slices) break;
            const uint32_t c = cnt[b], p = run;
            run += pad4(c);
            cnt[b] = p;
            for (uint32_t x = p + c; x < run; ++x) sorted[x] = 1u << sl;   // padding: the slice's sentinel bit
        }
        uint32_t total = 0;
        for (uint32_t q = 0; q < kRunThreads / 64; ++q) total += wsum[q];
        __syncthreads();
        // Run starts, in 4-entry chunks, to the subgroup's row of the table
        // (live counts zero until the lookup writes them).
        uint32_t *trow = table + (size_t)s * (PG.n_slices + 1);
        for (uint32_t b = t; b < PG.n_slices; b += kRunThreads) trow[b] = cnt[b] >> 2;
        if (t == 0) trow[PG.n_slices] = total >> 2;
        __syncthreads();

        // Placement: each VAT's entry (host within subgroup, AT within slice)
        // at its slice's cursor.
        if (wave_host) {
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                const uint32_t host = host_w + j * PG.dq;
                if (host < nh) {
                    const uint32_t slot = atomicAdd(&cnt[pid[j] >> sl], 1u);
                    sorted[slot] = (host << (sl + 1)) | (pid[j] & mask);
                }
            }
        } else if (PG.dr == 0) {
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j)
                if (t + j * kRunThreads < nv) {
                    const uint32_t slot = atomicAdd(&cnt[pid[j] >> sl], 1u);
                    sorted[slot] = ((host_t + j * PG.dq) << (sl + 1)) | (pid[j] & mask);
                }
        } else {
            uint32_t host = host_t, i = i_t;
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                if (t + j * kRunThreads < nv) {
                    const uint32_t slot = atomicAdd(&cnt[pid[j] >> sl], 1u);
                    sorted[slot] = (host << (sl + 1)) | (pid[j] & mask);
                }
                const bool wrap = i + PG.dr >= G.g;
                i = i + PG.dr - (wrap ? G.g : 0u);
                host += PG.dq + (wrap ? 1u : 0u);
            }
        }
        __syncthreads();

        // Copy out as one coalesced stream.
        uint4 *out = reinterpret_cast<uint4 *>(entries + (size_t)s * PG.region);
        for (uint32_t q = t; q < total / 4; q += kRunThreads) out[q] = reinterpret_cast<const uint4 *>(sorted)[q];
        // Ready the next subgroup's counters: the copy above reads only the
        // sorted entries.
        for (uint32_t q = t; q < nsp; q += kRunThreads) cnt[q] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Component m of a 16-byte chunk, m in [0, 4).
__device__ __forceinline__ uint32_t comp4(const uint4 &v, uint32_t m)
{
    return m == 0 ? v.x : m == 1 ? v.y : m == 2 ? v.z : v.w;
}

constexpr uint32_t kBmLoads = 8;      // 16-byte bitmap loads in flight per thread
constexpr uint32_t kDistWords = 8;    // bitmap words whose first live AT is loaded together

// Rank support for the slice's activity bits in the lookup's LDS: the live
// ATs before each superblock of 2048 ATs (32 bits) and before each block of
// 256 ATs within its superblock (16 bits); a live AT's rank is those plus
// the set bits before it in its block's eight words.
constexpr uint32_t kBlkLog2 = 8, kSupLog2 = 11;

__device__ __forceinline__ uint32_t live_rank(const uint32_t *bm, const uint32_t *sup, const uint16_t *blk,
                                              uint32_t o)
{
    uint32_t r = sup[o >> kSupLog2] + blk[o >> kBlkLog2];
    const uint32_t w = o >> 5;
    for (uint32_t x = w & ~7u; x < w; ++x) r += __popc(bm[x]);
    return r + __popc(bm[w] & ((1u << (o & 31u)) - 1u));
}

template <int W>
__global__ void __launch_bounds__(kRunThreads) k_run_lookup(Geo G, PartGeo PG, const uint8_t *__restrict__ pool,
                                                           const uint32_t *__restrict__ bitmap,
                                                           const DevState *__restrict__ st,
                                                           const uint32_t *__restrict__ entries,
                                                           uint32_t *__restrict__ table, uint32_t *__restrict__ hits_out,
                                                           uint32_t *__restrict__ heads)
{
    // LDS: the slice's activity bits (then zero words up to a whole block and
    // the padding entries' sentinel word), the rank tables, one live-result
    // counter per run of each wavefront's window, and the distances of the
    // slice's live ATs in slice order (when they fit).
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ uint32_t wsum[kRunThreads / 64];
    const uint32_t sl = PG.sl, mask = (1u << sl) - 1u, omask = (2u << sl) - 1u;
    const uint32_t nw = PG.bm_words, nwp = PG.bm_words_lds;
    const uint32_t nblk = nwp / 8u, nsup = (nblk + 7u) / 8u;
    uint32_t *bm = lds;
    uint32_t *sup = bm + nwp;
    uint16_t *blk = reinterpret_cast<uint16_t *>(sup + nsup);
    uint32_t *rcnt = sup + nsup + (nblk + 1u) / 2u;
    uint8_t *dist8 = reinterpret_cast<uint8_t *>(rcnt + kRunThreads);
    uint16_t *dist16 = reinterpret_cast<uint16_t *>(dist8);

    uint32_t b, part;
    if (PG.xcd) {              // XCD x mod 8 takes a contiguous range of slices
        const uint32_t r = blockIdx.x & 7u, u = blockIdx.x >> 3;
        const uint32_t per = PG.n_slices / 8u;
        part = u % PG.split;
        b = r * per + u / PG.split;
    } else {
        part = blockIdx.x % PG.split;
        b = blockIdx.x / PG.split;
    }
    const uint32_t s_lo = part * PG.span, s_hi = min(PG.n_sub, s_lo + PG.span);
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    {
        // From 2^7 ATs a slice's words are whole 16-byte groups (16-byte
        // aligned): a thread issues all its group loads before it stores any,
        // so the slice's bits take one round trip rather than one per word.
        const uint32_t *src = bitmap + (size_t)b * nw;
        const uint32_t nv = sl >= 7 ? nw / 4u : 0u;
        const uint4 *src4 = reinterpret_cast<const uint4 *>(src);
        uint4 *bm4 = reinterpret_cast<uint4 *>(bm);
        for (uint32_t q0 = t; q0 < nv; q0 += kBmLoads * kRunThreads) {
            uint4 v[kBmLoads];
#pragma unroll
            for (uint32_t u = 0; u < kBmLoads; ++u) {
                const uint32_t q = q0 + u * kRunThreads;
                v[u] = src4[q < nv ? q : q0];     // a group past the end reloads q0 and is not stored
            }
            // every load is used here, so none is sunk into its store's branch
#pragma unroll
            for (uint32_t u = 0; u < kBmLoads; ++u) asm volatile("" ::"v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w));
#pragma unroll
            for (uint32_t u = 0; u < kBmLoads; ++u) {
                const uint32_t q = q0 + u * kRunThreads;
                if (q < nv) bm4[q] = v[u];
            }
        }
        for (uint32_t q = 4u * nv + t; q < nwp; q += kRunThreads) {
            uint32_t v = q < nw ? src[q] : 0u;
            if (sl < 5 && q == 0) v &= (1u << (1u << sl)) - 1u;   // bits past the pool: the sentinel among them
            bm[q] = v;
        }
    }
    __syncthreads();
    // rank tables: thread x < nsup sums its superblock's blocks
    uint32_t stot = 0;
    if (t < nsup) {
        for (uint32_t k = 0; k < 8u && 8u * t + k < nblk; ++k) {
            const uint32_t kb = 8u * t + k;
            blk[kb] = (uint16_t)stot;
            for (uint32_t x = 0; x < 8u; ++x) stot += __popc(bm[8u * kb + x]);
        }
    }
    // exclusive scan of the superblock totals (nsup <= kRunThreads)
    {
        uint32_t incl = stot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= (uint32_t)off) incl += y;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint32_t run = incl - stot;
        for (uint32_t q = 0; q < wv; ++q) run += wsum[q];
        if (t < nsup) sup[t] = run;
    }
    uint32_t live = 0;
    for (uint32_t q = 0; q < kRunThreads / 64; ++q) live += wsum[q];
    const uint32_t bact0 = st->bact0;
    const uint32_t inact = inactive_value(G);
    const uint32_t first = b << sl;      // b < 2^(c - sl): no overflow
    uint32_t act0 = 0, act1 = 0, split = 0;
    if (PG.fast) {             // the slice meets block bid0 and at most block bid0 + 1
        const uint32_t bid0 = block_of(G, first);
        act0 = block_act(G, bact0, bid0);
        const uint64_t nxt = block_start(G, bid0 + 1);
        split = nxt - first > (uint64_t)mask ? mask + 1u : (uint32_t)(nxt - first);
        act1 = block_act(G, bact0, bid0 + 1 < G.twok ? bid0 + 1 : bid0);
    }
    // Distance (Eq. 5) of a live AT at offset o of the slice, from the pool;
    // its bit says it is active for window k, so d < k.
    auto dist_of = [&](uint32_t o, uint32_t v) -> uint32_t {
        if (v == inact) return G.k;
        uint32_t d;
        if (G.dr) {
            d = v;
        } else {
            const uint32_t act = PG.fast ? (o < split ? act0 : act1) : block_act(G, bact0, block_of(G, first | o));
            d = at_dist(G, act, v);
        }
        return d < G.k ? d : G.k;
    };
    auto dist_at = [&](uint32_t o) -> uint32_t { return dist_of(o, load_at<W>(pool, first | o, G.wb)); };
    auto put_dist = [&](uint32_t r, uint32_t d) {
        if (PG.dist16) dist16[r] = (uint16_t)d; else dist8[r] = (uint8_t)d;
    };
    // The distances of the slice's live ATs, in slice order, when they fit
    // the LDS left over; otherwise each live entry reads its AT from the pool.
    // A thread takes a contiguous range of words: one rank lookup for its
    // first word, then running popcounts.  Words go kDistWords at a time;
    // the AT of each word's first live bit is loaded for all of them at once
    // (a word with no live bit loads the slice's first AT and drops it), and
    // a word's further live bits (a few per cent of the words) one by one.
    const bool in_lds = live <= PG.dist_cap;
    __syncthreads();
    if (in_lds) {
        const uint32_t per = (nw + kRunThreads - 1u) / kRunThreads;
        const uint32_t q_lo = min(nw, t * per), q_hi = min(nw, q_lo + per);
        uint32_t r = q_lo < q_hi ? live_rank(bm, sup, blk, 32u * q_lo) : 0u;
        for (uint32_t q0 = q_lo; q0 < q_hi; q0 += kDistWords) {
            uint32_t bits[kDistWords], v[kDistWords], rb[kDistWords];
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u) {
                // q < q_hi + 7 <= nw + 7 stays inside the LDS block (the
                // rank tables follow the bits); words past q_hi count as empty
                const uint32_t q = q0 + u, w = bm[q];
                bits[u] = q < q_hi ? w : 0u;
            }
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u) {
                const uint32_t o = bits[u] ? 32u * (q0 + u) + (uint32_t)__builtin_ctz(bits[u]) : 0u;
                v[u] = load_at<W>(pool, first | o, G.wb);
            }
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u) asm volatile("" : "+v"(v[u]));
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u) {
                rb[u] = r;
                r += (uint32_t)__popc(bits[u]);
            }
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u)
                if (bits[u]) put_dist(rb[u], dist_of(32u * (q0 + u) + (uint32_t)__builtin_ctz(bits[u]), v[u]));
#pragma unroll
            for (uint32_t u = 0; u < kDistWords; ++u) {
                uint32_t rest = bits[u] & (bits[u] - 1u), rr = rb[u] + 1u;
                while (rest) {
                    const uint32_t x = __builtin_ctz(rest);
                    rest &= rest - 1u;
                    put_dist(rr++, dist_at(32u * (q0 + u) + x));
                }
            }
        }
    }
    __syncthreads();

    const uint32_t row = PG.n_slices + 1;
    uint16_t *tab16 = reinterpret_cast<uint16_t *>(table);
    const uint4 *ent4 = reinterpret_cast<const uint4 *>(entries);
    const uint32_t rq = PG.region / 4;
    constexpr uint32_t kPass = 64u * kLookU;
    uint32_t *cnt = rcnt + 64u * wv;
    // A lane's chunks of a pass and their runs.  A chunk past the end of the
    // flat list keeps the entries it held before (the padding sentinel at
    // first, every offset in range of the slice's bits); its bits are masked.
    uint4 e4[kLookU];
    uint32_t jr[kLookU];
#pragma unroll
    for (uint32_t q = 0; q < kLookU; ++q) {
        const uint32_t pad = 1u << sl;
        e4[q] = make_uint4(pad, pad, pad, pad);
        jr[q] = 0;
    }
    // A wavefront takes windows of 64 subgroups (lane r: run r of the
    // window), kRunThreads subgroups apart.  The window's runs in this slice
    // are one flat list of chunks (run after run), read in passes of kLookU
    // chunks per lane.  A live entry takes the next slot of its run from an
    // LDS counter (the order within a run is immaterial: the finalize only
    // counts), and its distance from LDS.
    for (uint32_t s0 = s_lo + wv * 64u; s0 < s_hi; s0 += kRunThreads) {
        uint32_t Sv = 0, len = 0;      // lane r: start (chunks) and length of run r
        if (lane < s_hi - s0) {
            const size_t cell = (size_t)(s0 + lane) * row + b;
            Sv = tab16[2 * cell];
            len = (uint32_t)tab16[2 * cell + 2] - Sv;
        }
        cnt[lane] = 0;
        uint32_t incl = len;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= (uint32_t)off) incl += y;
        }
        const uint32_t Fv = incl - len;                         // run r's first chunk in the flat list
        const uint32_t Ftot = __builtin_amdgcn_readlane(incl, 63);
        // chunk i of the flat list, in run r, is chunk Bv + i of the entries
        // (mod 2^32; the planner keeps every chunk index below 2^32)
        const uint32_t Bv = (s0 + lane) * rq + Sv - Fv;
        for (uint32_t base = 0; base < Ftot; base += kPass) {
#pragma unroll
            for (uint32_t q = 0; q < kLookU; ++q) {
                const uint32_t i0 = base + 64u * q, i = i0 + lane;
                if (i0 < Ftot) {
                    // run of chunk i: the last r with F_r <= i (F is nondecreasing,
                    // and an empty run shares its F with the next)
                    const uint32_t last = min(i0 + 63u, Ftot - 1u);
                    const uint32_t jb = (uint32_t)__popcll(__ballot(Fv <= i0)) - 1u;
                    const uint32_t je = (uint32_t)__popcll(__ballot(Fv <= last)) - 1u;
                    uint32_t j = jb, Bj = __builtin_amdgcn_readlane(Bv, jb);
                    for (uint32_t jj = jb + 1; jj <= je; ++jj) {
                        const uint32_t f = __builtin_amdgcn_readlane(Fv, jj);
                        const uint32_t bj = __builtin_amdgcn_readlane(Bv, jj);
                        if (i >= f) j = jj, Bj = bj;
                    }
                    jr[q] = j;
                    if (i < Ftot) e4[q] = ent4[Bj + i];
                }
            }
            // live bits (CheckAT for window k); a padding entry reads the
            // zero sentinel bit
            uint32_t M = 0;
#pragma unroll
            for (uint32_t q = 0; q < kLookU; ++q)
#pragma unroll
                for (uint32_t m = 0; m < 4; ++m) {
                    const uint32_t o = comp4(e4[q], m) & omask;
                    M |= __builtin_amdgcn_ubfe(bm[o >> 5], o, 1u) << (4u * q + m);   // bit o mod 32
                }
            // chunks past the list's end hold entries of an earlier pass
            if (base + kPass > Ftot) {
#pragma unroll
                for (uint32_t q = 0; q < kLookU; ++q)
                    if (base + 64u * q + lane >= Ftot) M &= ~(0xFu << (4u * q));
            }
            // the live entries, up to four per lane per round (every lane
            // takes part in the shuffles)
            while (__ballot(M != 0)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r > 0 && !__ballot(M != 0)) break;   // a round only while some lane has one left
                    const bool ok = M != 0;
                    const uint32_t p = ok ? (uint32_t)__builtin_ctz(M) : 0u;
                    if (ok) M &= M - 1u;
                    const uint32_t q = p >> 2, m = p & 3u;
                    uint4 c4 = e4[0];
                    uint32_t j = jr[0];
#pragma unroll
                    for (uint32_t qq = 1; qq < kLookU; ++qq)
                        if (q == qq) c4 = e4[qq], j = jr[qq];
                    const uint32_t Sj = __shfl(Sv, (int)j, 64);
                    if (ok) {
                        const uint32_t e = comp4(c4, m), o = e & mask;
                        const uint32_t d = in_lds ? (PG.dist16 ? (uint32_t)dist16[live_rank(bm, sup, blk, o)]
                                                               : (uint32_t)dist8[live_rank(bm, sup, blk, o)])
                                                  : dist_at(o);
                        const uint32_t slot = atomicAdd(&cnt[j], 1u);
                        const uint32_t val = ((e >> (sl + 1)) << 16) | d;
                        if (slot < 4u)
                            heads[((size_t)(s0 + j) * PG.n_slices + b) * 4u + slot] = val;
                        else
                            hits_out[(size_t)(s0 + j) * PG.region + 4u * Sj + (slot - 4u)] = val;
                    }
                }
            }
        }
        // live count of each run beside its start
        if (lane < s_hi - s0) tab16[2 * ((size_t)(s0 + lane) * row + b) + 1] = (uint16_t)cnt[lane];
    }
}

// ---------------------------------------------------------------------------
enum FinMode { kFinClosedForm = 0, kFinMulti = 1, kFinLearned = 2 };

// Several windows from one pass (ascending k' values).
constexpr uint32_t kMaxWindows = 64;

struct Windows {
    uint32_t m;
    uint32_t kp[kMaxWindows];
};

__device__ __forceinline__ uint32_t hist_bin(const uint32_t *row, uint32_t d)
{
    return (row[d >> 1] >> ((d & 1u) << 4)) & 0xFFFFu;
}

// The learned estimate (window k) of n16 <= 16 hosts by one whole wavefront:
// features from their packed histogram rows (LDS, stride rowp), live counts
// and closed forms (LDS, 16 each), the network on the matrix cores, exp of
// its output (the closed form where that is not finite) to est[0, n16).
// Each wavefront works on its own 16 rows and synchronizes only with itself.
// Returns the hosts given the closed form (the same in every lane).
// geo_off: the envelope rules the network out for this sketch's geometry
// (the same for every host; read once by the caller).
__device__ __forceinline__ uint32_t learned16(const Geo &G, float occupancy, const uint32_t *rw, uint32_t rowp,
                                          uint32_t n16, const float *cf16, const uint32_t *live16, uint16_t *xs,
                                          uint16_t *a1, const mlp::Packed *__restrict__ P, float *__restrict__ est,
                                          bool geo_off)
{
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const float fg = (float)G.g;
    // x / g as a product when g is a power of two (then exactly equal)
    const bool g_pow2 = (G.g & (G.g - 1u)) == 0u;
    const float inv_g = 1.0f / fg;
    // Row m (host m) is built by the whole wavefront, lane f = feature f, so
    // one ballot per row says whether the host is outside the envelope.
    uint32_t outside = geo_off ? 0xFFFFu : 0u;
    const mlp::EnvRange rng = mlp::env_range(P, l);     // this lane's feature in every row
    // ln(max(closed form, 1)) and the live count of host l mod 16, once per lane
    const float lnc = logf(fmaxf(cf16[l & 15], 1.0f));
    const uint32_t lvl = live16[l & 15];
    // Lane f builds feature f of every row, branch-free: every lane reads a
    // word of the row (the bins' word for f < k, a word of the row otherwise)
    // and keeps what its feature needs; rows past n16 read row 0 and are
    // zeroed.
    const int f = l;
    const bool f_hist = f < (int)G.k, f_live = f == (int)G.k;
    const bool f_occ = f == (int)G.k + 1, f_ln = f == (int)G.k + 2;
    const uint32_t hw = min((uint32_t)f >> 1, rowp - 1u), hs = ((uint32_t)f & 1u) << 4;
    static_assert(VATE_MLP_FEATURES == 64, "one feature per lane");
    // four rows at a time: their words are read together, in every lane
#pragma unroll
    for (uint32_t m0 = 0; m0 < 16; m0 += 4) {
        uint32_t hv[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) hv[u] = rw[(m0 + u < n16 ? m0 + u : 0u) * rowp + hw];
        asm volatile("" : "+v"(hv[0]), "+v"(hv[1]), "+v"(hv[2]), "+v"(hv[3]));
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t m = m0 + u;
            const float lnm = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(lnc), m));
            const uint32_t lv = __builtin_amdgcn_readlane(lvl, m);
            float x = (float)((hv[u] >> hs) & 0xFFFFu);
            x = f_hist ? x : (f_live ? (float)lv : 0.f);
            x = g_pow2 ? x * inv_g : x / fg;
            x = f_occ ? occupancy : (f_ln ? lnm * 0.0625f : x);
            if (m >= n16) x = 0.f;
            const uint16_t xb = mlp::bf16_bits(x);
            xs[m * mlp::LDS_STRIDE + f] = xb;
            if (__ballot(mlp::env_outside(rng, xb))) outside |= 1u << m;
        }
    }
    mlp::wave_sync();
    float r4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) r4[r] = __shfl(lnc, 4 * q + r, 64);
    mlp::f32x4 z1[4], z2[4];
    float a2v[4][4], o4[4];
    mlp::forward16<false>(P, xs, a1, r4, z1, z2, a2v, o4);
    bool fell = false;
    if (c < 4) {
        const uint32_t m = 4 * q + c;
        if (m < n16) {
            const float ex = expf(o4[c]);
            fell = ((outside >> m) & 1u) || !isfinite(ex);
            est[m] = fell ? cf16[m] : ex;
        }
    }
    return (uint32_t)__popcll(__ballot(fell));
}

// At least 5 wavefronts per SIMD: the network's registers would otherwise
// hold the streaming pass to 4 (measured 0.64 against 0.58 ms on the 40G
// workload; 6 would spill).
constexpr uint32_t kFinRuns = 4;   // runs whose cells a finalize thread loads together

template <int MODE>
__global__ void __launch_bounds__(kFinThreads, 5) k_run_finalize(Geo G, PartGeo PG, const DevState *__restrict__ st,
                                                             uint32_t n, uint32_t kprime,
                                                             const uint32_t *__restrict__ hits,
                                                             const uint32_t *__restrict__ heads,
                                                             const uint32_t *__restrict__ table, float *__restrict__ est,
                                                             uint32_t *__restrict__ live_out,
                                                             uint32_t *__restrict__ hist_out, Windows win,
                                                             const unsigned long long *__restrict__ cum,
                                                             const mlp::Packed *__restrict__ P,
                                                             float *__restrict__ cf_out)
{
    // [hosts][rowp] packed 16-bit bins of the workgroup's fgroup subgroups
    extern __shared__ __attribute__((aligned(16))) uint32_t hist[];
    const uint32_t t = threadIdx.x;
    const uint32_t s0 = blockIdx.x * PG.fgroup;
    const uint32_t nsg = min(PG.fgroup, PG.n_sub - s0);
    const uint32_t h0 = s0 * PG.hosts;
    const uint32_t nh = min(nsg * PG.hosts, n - h0);
    const uint32_t rowp = PG.rowp;
    const uint32_t ns = PG.n_slices, nr = nsg * ns;
    for (uint32_t q = t; q < nh * rowp; q += kFinThreads) hist[q] = 0;
    __syncthreads();
    {
        // Live results (host within its subgroup << 16 | distance) of run r
        // (slice r mod n_slices of subgroup s0 + r / n_slices): the first
        // four in the run's 16-byte cell of `heads`, any more in the run's
        // own result slots.  Each is counted into its host's bin with an LDS
        // atomic; bin k (inactive) is not counted: it is g minus the others,
        // filled in below.  (A live count never exceeds the run's entries;
        // the clamp keeps every read inside them whatever the table holds.)
        // A thread takes kFinRuns runs at a time: their table cells and head
        // cells are all loaded before the first is counted (one round trip
        // for the batch; a run past the end reloads the batch's first run's
        // cells and is skipped, a run without live results ignores its head).
        const uint4 *heads4 = reinterpret_cast<const uint4 *>(heads);
        for (uint32_t r0 = t; r0 < nr; r0 += kFinRuns * kFinThreads) {
            uint32_t c[kFinRuns], c1[kFinRuns];
            uint4 w4[kFinRuns];
#pragma unroll
            for (uint32_t u = 0; u < kFinRuns; ++u) {
                const uint32_t r = r0 + u * kFinThreads < nr ? r0 + u * kFinThreads : r0;
                const uint32_t sg = r / ns, b = r - sg * ns;
                const uint32_t *trow = table + (size_t)(s0 + sg) * (ns + 1);
                c[u] = trow[b];
                c1[u] = trow[b + 1];
                w4[u] = heads4[(size_t)(s0 + sg) * ns + b];
            }
            // every load is used here, so none is sunk into its run's branch
#pragma unroll
            for (uint32_t u = 0; u < kFinRuns; ++u)
                asm volatile("" ::"v"(c[u]), "v"(c1[u]), "v"(w4[u].x), "v"(w4[u].y), "v"(w4[u].z), "v"(w4[u].w));
#pragma unroll
            for (uint32_t u = 0; u < kFinRuns; ++u) {
                const uint32_t r = r0 + u * kFinThreads;
                if (r >= nr) break;
                const uint32_t sg = r / ns;
                const uint32_t start = c[u] & 0xFFFFu;
                const uint32_t cnt = min(c[u] >> 16, 4u * ((c1[u] & 0xFFFFu) - start));
                const uint32_t hrow = sg * PG.hosts;
#pragma unroll
                for (uint32_t m = 0; m < 4; ++m) {
                    if (m >= cnt) break;
                    const uint32_t v = comp4(w4[u], m), d = v & 0xFFFFu;
                    if (d < G.k) atomicAdd(&hist[(hrow + (v >> 16)) * rowp + (d >> 1)], 1u << ((d & 1u) << 4));
                }
                const uint32_t *more = hits + (size_t)(s0 + sg) * PG.region + 4u * start;
                for (uint32_t i = 4; i < cnt; ++i) {
                    const uint32_t v = more[i - 4u], d = v & 0xFFFFu;
                    if (d < G.k) atomicAdd(&hist[(hrow + (v >> 16)) * rowp + (d >> 1)], 1u << ((d & 1u) << 4));
                }
            }
        }
    }
    __syncthreads();
    if (MODE == kFinClosedForm && hist_out) {   // only the histogram output has bin k
        for (uint32_t h = t; h < nh; h += kFinThreads) {   // bin k = g - (bins 0 .. k-1)
            uint32_t *row = hist + h * rowp;
            uint32_t live = 0;
            for (uint32_t j = 0; j < G.k / 2; ++j) live += (row[j] & 0xFFFFu) + (row[j] >> 16);
            const uint32_t w = G.k >> 1;
            if (G.k & 1u) {
                live += row[w] & 0xFFFFu;
                row[w] = (row[w] & 0xFFFFu) | ((G.g - live) << 16);
            } else {
                row[w] = G.g - live;
            }
        }
        __syncthreads();
    }

    if constexpr (MODE == kFinClosedForm) {
        const uint64_t active_pool = pool_active(st, kprime);
        for (uint32_t h = t; h < nh; h += kFinThreads) {
            const uint32_t *row = hist + h * rowp;
            uint32_t live = 0;
            for (uint32_t d = 0; d < kprime; ++d) live += hist_bin(row, d);
            est[h0 + h] = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
            if (live_out) live_out[h0 + h] = live;
        }
        if (hist_out) {
            const uint32_t kp1 = G.k + 1;
            uint32_t *out = hist_out + (size_t)h0 * kp1;
            for (uint32_t q = t; q < nh * kp1; q += kFinThreads) {
                const uint32_t h = q / kp1, d = q - h * kp1;
                out[q] = hist_bin(hist + h * rowp, d);
            }
        }
    } else if constexpr (MODE == kFinMulti) {
        for (uint32_t h = t; h < nh; h += kFinThreads) {
            const uint32_t *row = hist + h * rowp;
            float *e = est + (size_t)(h0 + h) * win.m;
            uint32_t live = 0, jw = 0;
            for (uint32_t d = 0; d < G.k && jw < win.m; ++d) {
                live += hist_bin(row, d);
                while (jw < win.m && win.kp[jw] == d + 1) {
                    e[jw] = estimate_from_counts(G.g - live, G.N - cum[d + 1], G.g, G.c);
                    ++jw;
                }
            }
        }
    } else {
        // Learned estimate, in groups of 64 hosts (16 per wavefront): the
        // closed form for window k, then the network fed from the LDS rows.
        // One 16-row staging tile per wavefront holds its features and then
        // its first layer's activations: the layer's inputs are in registers
        // (its products depend on them) before its outputs are written.
        __shared__ __attribute__((aligned(16))) uint16_t xs_all[kFinThreads / 64][16 * mlp::LDS_STRIDE];
        __shared__ float cf_s[kFinThreads / 4];
        __shared__ uint32_t live_s[kFinThreads / 4];
        const uint64_t active_pool = pool_active(st, G.k);
        const float occupancy = (float)active_pool / (float)G.N;
        const uint32_t w = t >> 6;
        const bool geo_off = mlp::env_geometry_off(P, G.k, G.g, G.c, G.wb);
        __shared__ uint32_t fell_wg;      // the workgroup's fallback hosts (one counter atomic per workgroup)
        if (t == 0) fell_wg = 0;
        __syncthreads();                  // (the loop below synchronizes wavefronts only with themselves)
        uint32_t fell_wave = 0;
        for (uint32_t base = 0; base < nh; base += kFinThreads / 4) {
            {   // live count and closed form of host base + t / 4, four threads a host
                const uint32_t hh = t >> 2, qq = t & 3u;
                uint32_t live = 0;
                if (base + hh < nh) {
                    const uint32_t *row = hist + (base + hh) * rowp;
                    for (uint32_t j = qq; j < G.k / 2; j += 4) live += (row[j] & 0xFFFFu) + (row[j] >> 16);
                    if (qq == 0 && (G.k & 1u)) live += row[G.k / 2] & 0xFFFFu;
                }
                live += __shfl_xor(live, 1, 64);
                live += __shfl_xor(live, 2, 64);
                if (qq == 0) {
                    float cf = 0.f;
                    if (base + hh < nh) {
                        cf = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
                        cf_out[h0 + base + hh] = cf;
                    }
                    cf_s[hh] = cf;
                    live_s[hh] = live;
                }
            }
            mlp::wave_sync();   // hosts 16 w .. 16 w + 15 are wavefront w's, here and below
            const uint32_t m0 = base + 16 * w;
            const uint32_t n16 = nh > m0 ? min(16u, nh - m0) : 0u;
            // An opaque zero offset per group, so the weight fragments are
            // loaded where they are used rather than hoisted out of the loop
            // into registers (the pointer stays a global one, so the loads
            // are global loads that wait only on the vector-memory counter).
            uint32_t zero = 0;
            asm volatile("" : "+s"(zero));
            const mlp::Packed *Pg = P + zero;
            fell_wave += learned16(G, occupancy, hist + m0 * rowp, rowp, n16, cf_s + 16 * w, live_s + 16 * w,
                                   xs_all[w], xs_all[w], Pg, est + h0 + m0, geo_off);
            mlp::wave_sync();
        }
        if ((t & 63u) == 0 && fell_wave) atomicAdd(&fell_wg, fell_wave);
        __syncthreads();
        if (t == 0) mlp::env_count(P, fell_wg);
    }
}

// Per-host windows from full histograms in memory (the fallback when the
// partitioned lookups are not available for a geometry).
__global__ void k_multi_from_hist(Geo G, uint32_t n, Windows win, const unsigned long long *__restrict__ cum,
                                  const uint32_t *__restrict__ hist, float *__restrict__ est)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    const uint32_t *row = hist + (size_t)h * (G.k + 1);
    uint32_t live = 0, j = 0;
    for (uint32_t d = 0; d < G.k && j < win.m; ++d) {
        live += row[d];
        while (j < win.m && win.kp[j] == d + 1) {
            est[(size_t)h * win.m + j] = estimate_from_counts(G.g - live, G.N - cum[d + 1], G.g, G.c);
            ++j;
        }
    }
}

__global__ void k_census_prefix(Geo G, const DevState *__restrict__ st, unsigned long long *__restrict__ cum)
{
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        cum[0] = 0;
        for (uint32_t d = 0; d < G.k; ++d) {
            run += census_of(st)[d];
            cum[d + 1] = run;
        }
    }
}
