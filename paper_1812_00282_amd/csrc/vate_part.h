// Partitioned estimate: the g CheckAT lookups of every host (Alg. 4's
// estimate loop, Alg. 1) routed to the pool slice that holds their AT,
// resolved out of LDS, and routed back.  Included into vate.hip inside
// namespace vate.
//
// The direct gather reads one random cache line per VAT anywhere in the
// pool, so it is bound by line fills from beyond L2.  Here:
//
//  k_run_scatter  persistent workgroups, one subgroup of hosts at a time.
//                 Hashes the subgroup's VATs (their slices stay in
//                 registers), counts them per pool slice in LDS, places their
//                 16-bit indices by an LDS counting sort (two bytes a slot is
//                 what lets a subgroup hold 63 hosts of g = 1024), then
//                 copies the sorted entries (host within subgroup, AT within
//                 slice; the pid hashed again from the index) to the
//                 workspace as one coalesced stream.  Every (subgroup, slice)
//                 run starts on a 4-entry boundary (padded with kRunPad), so
//                 no 16-byte chunk is shared by two slices.  Run starts, in
//                 chunks, go to a u16 table laid out
//                 [super-slice][subgroup][slice in super].
//  k_run_lookup   one workgroup per pool slice (128 KiB of ATs, held in LDS).
//                 Walks that slice's run in every subgroup and writes, beside
//                 each entry, a 16-bit result: the host within the subgroup
//                 and the VAT's distance (Eq. 5, CheckAT; k = inactive for
//                 window k).  The 8 slices of a super-slice are given
//                 to one XCD: their runs are adjacent in memory, so the lines
//                 they read and the distance bytes they write meet in that
//                 XCD's L2.  Each slice's walk is split over kLookupSplit
//                 workgroups (ranges of subgroups).
//  k_run_finalize one workgroup per subgroup.  Streams the results back,
//                 builds each host's distance histogram in LDS and forms
//                 Eq. 11 for k', several windows, or the learned estimate
//                 (the network fed from the LDS histograms, 16 hosts per
//                 wavefront).
//
// HBM traffic per VAT: 4 B entry written and read back once, 2 B result
// written and read back once.

constexpr uint32_t kRunThreads = 1024;                          // scatter / lookup workgroup
constexpr uint32_t kRunPerThread = 64;                          // VATs hashed per scatter thread
constexpr uint32_t kRunMaxEntries = 65535;                      // VATs per subgroup: 16-bit indices, one value spare
constexpr uint32_t kSortPad = 0xFFFFu;                          // padding slot of the LDS sort
constexpr uint32_t kRunLdsMax = 160u * 1024u;                   // gfx950 LDS per workgroup
constexpr uint32_t kRunLdsStatic = 64u;                         // k_run_scatter's static LDS (wsum)
constexpr uint32_t kSliceBytesLog2 = 17;                        // pool bytes per slice: 128 KiB
constexpr uint32_t kRunMaxSlices = 8192;                        // pools up to 1 GiB
constexpr uint32_t kRunMaxHosts = 1024;                         // hosts per subgroup
constexpr uint32_t kRunPad = 0xFFFFFFFFu;                       // padding entry (never a real one: <= 28 bits)
constexpr uint32_t kSuper = 8;                                  // slices per super-slice
constexpr uint32_t kFinThreads = 256;
constexpr uint32_t kLookupSplit = 2;                            // subgroup ranges per slice (lookup)
constexpr uint32_t kLanesPerRun = 16;                           // lookup lanes per run, one 16-byte chunk each
constexpr uint32_t kRunsPerStep = 64 / kLanesPerRun;            // runs per wavefront step
constexpr uint32_t kSubPerWave = 8 * kRunsPerStep;              // subgroups per wavefront per pipeline stage
constexpr uint32_t kFinHistBytes = 64u * 1024u;                 // per-subgroup histogram ceiling

struct PartGeo {
    uint32_t sl;          // ATs per slice = 2^sl
    uint32_t n_slices;    // N >> sl
    uint32_t sub;         // slices per super-slice, min(8, n_slices)
    uint32_t n_super;     // n_slices / sub
    uint32_t hosts;       // hosts per subgroup
    uint32_t n_sub;       // subgroups
    uint32_t vats;        // hosts * g
    uint32_t cap;         // padded entries per subgroup at most: vats + 3 n_slices, rounded up to 4
    uint32_t region;      // entries between subgroup regions (cap rounded up to 64)
    uint32_t dq, dr;      // kRunThreads = dq * g + dr
    uint32_t fast;        // every block holds >= 2^sl ATs: a slice meets at most two blocks
    uint32_t rowp;        // u32 words per packed 16-bit histogram row: ceil((k + 1) / 2), made odd
    uint32_t xcd;         // map the slices of a super-slice to one XCD
    uint32_t split;       // lookup workgroups per slice, each over a range of subgroups
    uint32_t span;        // subgroups per range (a multiple of 1024)
    uint32_t lds_scatter, lds_lookup, lds_final;
    uint32_t dbits;       // distance bits of a result: values 0..k, all ones = padding
    uint32_t gmul;        // ceil(2^32 / g), v / g = umulhi(v, gmul) for v < 2^16; 0 for g = 1
};

// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pad4(uint32_t x) { return (x + 3u) & ~3u; }

__global__ void __launch_bounds__(kRunThreads) k_run_scatter(Geo G, PartGeo PG, const uint32_t *__restrict__ hosts,
                                                            uint32_t n, uint32_t *__restrict__ entries,
                                                            uint16_t *__restrict__ table)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ uint32_t wsum[kRunThreads / 64];
    const uint32_t nsp = (PG.n_slices + 3u) & ~3u;
    const uint32_t nkp = (PG.hosts + 3u) & ~3u;
    uint32_t *cnt = lds;                  // per-slice counts, then cursors
    uint32_t *keys = lds + nsp;           // host keys
    uint16_t *sorted = reinterpret_cast<uint16_t *>(keys + nkp);   // VAT indices by slice, runs padded to 4
    const uint32_t t = threadIdx.x;
    const uint32_t mask = (1u << PG.sl) - 1u;
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

        // VAT v = t + j * kRunThreads of the subgroup is VAT i = v mod g of
        // host v / g.  H's multiplier i * phi is carried along (mod 2^32);
        // when g divides the workgroup size, i (and i * phi) stay fixed and
        // only the host advances.  Iterations j < jfull are full for every
        // thread (a uniform branch); the ragged tail is iteration jfull.
        // H(aip, i) = top c bits of the mix (shift = 32 - c is at most 31).
        const uint32_t jfull = nv / kRunThreads, tail = nv - jfull * kRunThreads;
        uint32_t bs[kRunPerThread / 2];    // slices of the thread's VATs, two 16-bit values per word
#pragma unroll
        for (uint32_t j = 0; j < kRunPerThread / 2; ++j) bs[j] = 0;
        if (PG.dr == 0) {
            const uint32_t ik = i_t * kPhi;
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                const uint32_t host = host_t + j * PG.dq;
                if (j < jfull || (j == jfull && t < tail)) {
                    const uint32_t b = (mix(keys[host] ^ ik) >> G.shift) >> PG.sl;
                    bs[j >> 1] |= b << ((j & 1u) << 4);
                    atomicAdd(&cnt[b], 1u);
                }
            }
        } else {
            uint32_t host = host_t, i = i_t, ik = i_t * kPhi;
#pragma unroll
            for (uint32_t j = 0; j < kRunPerThread; ++j) {
                if (j < jfull || (j == jfull && t < tail)) {
                    const uint32_t b = (mix(keys[host] ^ ik) >> G.shift) >> PG.sl;
                    bs[j >> 1] |= b << ((j & 1u) << 4);
                    atomicAdd(&cnt[b], 1u);
                }
                const bool wrap = i + PG.dr >= G.g;
                i = i + PG.dr - (wrap ? G.g : 0u);
                ik = ik + d_ik - (wrap ? g_ik : 0u);
                host += PG.dq + (wrap ? 1u : 0u);
            }
        }
        __syncthreads();

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
            for (uint32_t x = p + c; x < run; ++x) sorted[x] = kSortPad;
        }
        uint32_t total = 0;
        for (uint32_t q = 0; q < kRunThreads / 64; ++q) total += wsum[q];
        __syncthreads();
        // Run starts to the table in 4-entry chunks, one 16-byte
        // (super-slice, subgroup) cell per store.
        if (PG.sub == kSuper) {
            for (uint32_t B = t; B < PG.n_super; B += kRunThreads) {
                const uint32_t *c8 = cnt + 8u * B;
                reinterpret_cast<uint4 *>(table)[(size_t)B * PG.n_sub + s] =
                    make_uint4((c8[0] >> 2) | ((c8[1] >> 2) << 16), (c8[2] >> 2) | ((c8[3] >> 2) << 16),
                               (c8[4] >> 2) | ((c8[5] >> 2) << 16), (c8[6] >> 2) | ((c8[7] >> 2) << 16));
            }
        } else {
            for (uint32_t b = t; b < PG.n_slices; b += kRunThreads)
                table[((size_t)(b / PG.sub) * PG.n_sub + s) * PG.sub + b % PG.sub] = (uint16_t)(cnt[b] >> 2);
        }
        if (t == 0) table[((size_t)PG.n_super * PG.n_sub + s) * PG.sub] = (uint16_t)(total >> 2);
        __syncthreads();

#pragma unroll
        for (uint32_t j = 0; j < kRunPerThread; ++j)
            if (j < jfull || (j == jfull && t < tail)) {
                const uint32_t slot = atomicAdd(&cnt[(bs[j >> 1] >> ((j & 1u) << 4)) & 0xFFFFu], 1u);
                sorted[slot] = (uint16_t)(t + j * kRunThreads);
            }
        __syncthreads();

        // Copy out, one 4-entry chunk per thread and step: each VAT index
        // becomes its entry (host within subgroup, AT within slice), its pid
        // hashed again (v / g by a multiply-high: exact for v, g < 2^16).
        uint4 *out = reinterpret_cast<uint4 *>(entries + (size_t)s * PG.region);
        for (uint32_t q = t; q < total / 4; q += kRunThreads) {
            const uint2 v2 = reinterpret_cast<const uint2 *>(sorted)[q];
            const uint32_t v[4] = {v2.x & 0xFFFFu, v2.x >> 16, v2.y & 0xFFFFu, v2.y >> 16};
            uint32_t e[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t host = PG.gmul ? __umulhi(v[m], PG.gmul) : v[m], i = v[m] - host * G.g;
                const uint32_t pid_m = mix(keys[min(host, PG.hosts - 1u)] ^ (i * kPhi)) >> G.shift;
                e[m] = v[m] == kSortPad ? kRunPad : (host << PG.sl) | (pid_m & mask);
            }
            out[q] = make_uint4(e[0], e[1], e[2], e[3]);
        }
        // Ready the next subgroup: the copy above reads only the sorted
        // indices and the keys, so both wait for the barrier.
        for (uint32_t q = t; q < nsp; q += kRunThreads) cnt[q] = 0;
        __syncthreads();
        if (t < nh_next) keys[t] = host_key(G, aip_next);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
template <typename DT>
__device__ __forceinline__ void store4(DT *p, const uint32_t d[4])
{
    if constexpr (sizeof(DT) == 1)
        *reinterpret_cast<uint32_t *>(p) = d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24);
    else
        *reinterpret_cast<uint2 *>(p) = make_uint2(d[0] | (d[1] << 16), d[2] | (d[3] << 16));
}

template <int W>
__global__ void __launch_bounds__(kRunThreads) k_run_lookup(Geo G, PartGeo PG, const uint8_t *__restrict__ pool,
                                                           const DevState *__restrict__ st,
                                                           const uint32_t *__restrict__ entries,
                                                           const uint16_t *__restrict__ table,
                                                           uint16_t *__restrict__ res)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const uint8_t *at = reinterpret_cast<const uint8_t *>(lds);
    uint32_t B, j;
    uint32_t part;                                  // subgroup range of this workgroup
    if (PG.xcd) {              // workgroup x runs on XCD x mod 8
        const uint32_t r = blockIdx.x & 7u, rest = blockIdx.x >> 3;
        j = rest % PG.sub;
        const uint32_t rest2 = rest / PG.sub;
        part = rest2 % PG.split;
        B = (rest2 / PG.split) * 8u + r;
    } else {
        j = blockIdx.x % PG.sub;
        const uint32_t rest2 = blockIdx.x / PG.sub;
        part = rest2 % PG.split;
        B = rest2 / PG.split;
    }
    const uint32_t s_lo = part * PG.span, s_hi = min(PG.n_sub, s_lo + PG.span);
    const uint32_t b = B * PG.sub + j;
    const uint32_t sl = PG.sl, mask = (1u << sl) - 1u;
    const uint32_t nbytes = (uint32_t)(((uint64_t)(W ? W : G.wb) << sl) >> 3);
    const uint8_t *src = pool + (uint64_t)b * nbytes;
    if ((nbytes & 15u) == 0) {
        for (uint32_t q = threadIdx.x; q < nbytes / 16; q += kRunThreads)
            reinterpret_cast<uint4 *>(lds)[q] = reinterpret_cast<const uint4 *>(src)[q];
    } else {
        for (uint32_t q = threadIdx.x; q < nbytes; q += kRunThreads)
            reinterpret_cast<uint8_t *>(lds)[q] = src[q];
    }
    __syncthreads();

    const uint32_t bact0 = st->bact0;
    const uint32_t inact = inactive_value(G);
    const uint32_t first = b << sl;
    uint32_t act0 = 0, act1 = 0, split = 0;
    if (PG.fast) {             // the slice meets block bid0 and at most block bid0 + 1
        const uint32_t bid0 = block_of(G, first);
        act0 = block_act(G, bact0, bid0);
        const uint64_t nxt = block_start(G, bid0 + 1);
        split = nxt - first > (uint64_t)mask ? mask + 1u : (uint32_t)(nxt - first);
        act1 = block_act(G, bact0, bid0 + 1 < G.twok ? bid0 + 1 : bid0);
    }
    auto dist_of = [&](uint32_t local) -> uint32_t {
        const uint32_t v = load_at<W>(at, local, G.wb);
        if (v == inact) return G.k;
        uint32_t d;
        if (G.dr) {
            d = v;
        } else {
            const uint32_t act = PG.fast ? (local < split ? act0 : act1)
                                         : block_act(G, bact0, block_of(G, first | local));
            d = at_dist(G, act, v);
        }
        return d < G.k ? d : G.k;
    };

    // kLanesPerRun lanes per subgroup run, four entries (one 16-byte chunk)
    // per lane.  A wavefront takes kSubPerWave subgroups at a time: one
    // coalesced read of their run bounds, then the first chunk of eight runs
    // per lane group is loaded before any is used (eight independent loads in
    // flight per lane); the rare chunks beyond a run's first kLanesPerRun
    // follow in a second pass.
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t grp = lane / kLanesPerRun, gl = lane % kLanesPerRun;
    const size_t row = (size_t)B * PG.n_sub, next_row = (size_t)(B + 1) * PG.n_sub;
    // Runs start and end on 4-entry boundaries: every chunk belongs to one
    // run.  A padding entry's result is all ones.
    auto resolve = [&](uint32_t s, uint32_t c, const uint4 &e4) {
        const uint32_t e[4] = {e4.x, e4.y, e4.z, e4.w};
        uint32_t r[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            r[m] = e[m] == kRunPad ? 0xFFFFu : (((e[m] >> sl) << PG.dbits) | dist_of(e[m] & mask));
        store4<uint16_t>(res + (size_t)s * PG.region + 4u * c, r);
    };
    // Software pipeline over groups of 64 subgroups: while group i is
    // resolved, the entries of group i + 1 and the run bounds of group i + 2
    // are already in flight.
    auto bounds = [&](uint32_t s0, uint32_t &st_l, uint32_t &en_l) {
        st_l = en_l = 0;
        if (lane < kSubPerWave && s0 + lane < s_hi) {
            const size_t cell = (row + s0 + lane) * PG.sub;
            st_l = table[cell + j];
            en_l = j + 1 < PG.sub ? table[cell + j + 1] : table[(next_row + s0 + lane) * PG.sub];
        }
    };
    auto issue = [&](uint32_t s0, uint32_t st_l, uint32_t en_l, uint4 e4[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t r = kRunsPerStep * q + grp;
            const uint32_t start = __shfl(st_l, (int)r, 64), end = __shfl(en_l, (int)r, 64);
            const uint32_t c = start + gl;
            e4[q] = make_uint4(0u, 0u, 0u, 0u);
            if (c < end) e4[q] = reinterpret_cast<const uint4 *>(entries + (size_t)(s0 + r) * PG.region)[c];
        }
    };
    auto finish = [&](uint32_t s0, uint32_t st_l, uint32_t en_l, const uint4 e4[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t r = kRunsPerStep * q + grp;
            const uint32_t start = __shfl(st_l, (int)r, 64), end = __shfl(en_l, (int)r, 64);
            const uint32_t c = start + gl;
            if (c < end) resolve(s0 + r, c, e4[q]);
        }
        // Chunks beyond a run's first kLanesPerRun, when any run of the
        // group has them (rare: runs average about a third of that).
        if (!__ballot(en_l - st_l > kLanesPerRun)) return;
        for (int q = 0; q < 8; ++q) {
            const uint32_t r = kRunsPerStep * q + grp;
            const uint32_t start = __shfl(st_l, (int)r, 64), end = __shfl(en_l, (int)r, 64);
            const uint32_t s = s0 + r, c1 = end;
            const uint4 *ent = reinterpret_cast<const uint4 *>(entries + (size_t)s * PG.region);
            for (uint32_t c = start + kLanesPerRun + gl;; c += kLanesPerRun) {
                const bool act = c < c1;
                if (!__ballot(act)) break;
                if (act) resolve(s, c, ent[c]);
            }
        }
    };
    const uint32_t step = (kRunThreads / 64) * kSubPerWave;   // 16 wavefronts
    uint32_t s0 = s_lo + wv * kSubPerWave;
    uint32_t stA, enA, stB, enB;
    uint4 eA[8];
    bounds(s0, stA, enA);
    issue(s0, stA, enA, eA);
    bounds(s0 + step, stB, enB);
    for (; s0 < s_hi; s0 += step) {
        uint4 eB[8];
        issue(s0 + step, stB, enB, eB);
        uint32_t stC, enC;
        bounds(s0 + 2 * step, stC, enC);
        finish(s0, stA, enA, eA);
#pragma unroll
        for (int q = 0; q < 8; ++q) eA[q] = eB[q];
        stA = stB, enA = enB, stB = stC, enB = enC;
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
// Every wavefront of the workgroup calls it (the network has a barrier).
__device__ __forceinline__ void learned16(const Geo &G, float occupancy, const uint32_t *rw, uint32_t rowp,
                                          uint32_t n16, const float *cf16, const uint32_t *live16, uint16_t *xs,
                                          uint16_t *a1, const mlp::Packed *__restrict__ P, float *__restrict__ est)
{
    const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
    const float fg = (float)G.g;
    for (int e = l; e < 16 * VATE_MLP_FEATURES; e += 64) {
        const int m = e >> 6, f = e & 63;
        float x = 0.f;
        if ((uint32_t)m < n16) {
            if (f < (int)G.k)
                x = (float)hist_bin(rw + m * rowp, f) / fg;
            else if (f == (int)G.k)
                x = (float)live16[m] / fg;
            else if (f == (int)G.k + 1)
                x = occupancy;
            else if (f == (int)G.k + 2)
                x = logf(fmaxf(cf16[m], 1.0f)) * 0.0625f;
        }
        xs[m * mlp::LDS_STRIDE + f] = mlp::bf16_bits(x);
    }
    __syncthreads();
    float r4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) r4[r] = logf(fmaxf(cf16[4 * q + r], 1.0f));
    mlp::f32x4 z1[4], z2[4];
    float a2v[4][4], o4[4];
    mlp::forward16(P, xs, a1, r4, z1, z2, a2v, o4);
    if (c < 4) {
        const uint32_t m = 4 * q + c;
        if (m < n16) {
            const float ex = expf(o4[c]);
            est[m] = isfinite(ex) ? ex : cf16[m];
        }
    }
}

// At least 5 wavefronts per SIMD: the network's registers would otherwise
// hold the streaming pass to 4 (measured 0.64 against 0.58 ms on the 40G
// workload; 6 would spill).
template <int MODE>
__global__ void __launch_bounds__(kFinThreads, 5) k_run_finalize(Geo G, PartGeo PG, const DevState *__restrict__ st,
                                                             uint32_t n, uint32_t kprime,
                                                             const uint16_t *__restrict__ res,
                                                             const uint16_t *__restrict__ table, float *__restrict__ est,
                                                             uint32_t *__restrict__ live_out,
                                                             uint32_t *__restrict__ hist_out, Windows win,
                                                             const unsigned long long *__restrict__ cum,
                                                             const mlp::Packed *__restrict__ P,
                                                             float *__restrict__ cf_out)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t hist[];   // [hosts][rowp] packed 16-bit bins
    const uint32_t s = blockIdx.x, t = threadIdx.x;
    const uint32_t h0 = s * PG.hosts;
    const uint32_t nh = min(PG.hosts, n - h0);
    const uint32_t nvp = 4u * table[((size_t)PG.n_super * PG.n_sub + s) * PG.sub];   // padded entries
    const uint32_t rowp = PG.rowp;
    for (uint32_t q = t; q < nh * rowp; q += kFinThreads) hist[q] = 0;
    __syncthreads();
    {
        const uint4 *rr = reinterpret_cast<const uint4 *>(res + (size_t)s * PG.region);   // 8 results per load
        const uint32_t dmask = (1u << PG.dbits) - 1u;
        constexpr uint32_t U = 8;     // loads in flight per thread
        const uint32_t nch = (nvp + 7u) >> 3;     // nvp is a multiple of 4
        for (uint32_t c0 = t; c0 < nch; c0 += U * kFinThreads) {
            uint4 r4[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t c = c0 + u * kFinThreads;
                if (c < nch) r4[u] = rr[c];
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t c = c0 + u * kFinThreads;
                if (c >= nch) break;
                const uint32_t w[4] = {r4[u].x, r4[u].y, r4[u].z, r4[u].w};
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    if (8u * c + m >= nvp) break;
                    // Bin k (inactive for window k, most of the VATs) and
                    // padding (d all ones) are not counted: bin k is g minus
                    // the others, filled in below.
                    const uint32_t r = (w[m >> 1] >> ((m & 1) << 4)) & 0xFFFFu;
                    const uint32_t d = r & dmask;
                    if (d >= G.k) continue;
                    atomicAdd(&hist[(r >> PG.dbits) * rowp + (d >> 1)], 1u << ((d & 1u) << 4));
                }
            }
        }
    }
    __syncthreads();
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
        __shared__ __attribute__((aligned(16))) uint16_t xs_all[kFinThreads / 64][16 * mlp::LDS_STRIDE];
        __shared__ __attribute__((aligned(16))) uint16_t a1_all[kFinThreads / 64][16 * mlp::LDS_STRIDE];
        __shared__ float cf_s[kFinThreads / 4];
        __shared__ uint32_t live_s[kFinThreads / 4];
        const uint64_t active_pool = pool_active(st, G.k);
        const float occupancy = (float)active_pool / (float)G.N;
        const uint32_t w = t >> 6;
        for (uint32_t base = 0; base < nh; base += kFinThreads / 4) {
            if (t < kFinThreads / 4) {
                uint32_t live = 0;
                float cf = 0.f;
                if (base + t < nh) {
                    const uint32_t *row = hist + (base + t) * rowp;
                    for (uint32_t j = 0; j < G.k / 2; ++j) live += (row[j] & 0xFFFFu) + (row[j] >> 16);
                    if (G.k & 1u) live += row[G.k / 2] & 0xFFFFu;
                    cf = estimate_from_counts(G.g - live, G.N - active_pool, G.g, G.c);
                    cf_out[h0 + base + t] = cf;
                }
                cf_s[t] = cf;
                live_s[t] = live;
            }
            __syncthreads();
            const uint32_t m0 = base + 16 * w;
            const uint32_t n16 = nh > m0 ? min(16u, nh - m0) : 0u;
            // Opaque per group, so the weight fragments are loaded where they
            // are used rather than hoisted out of the loop into registers.
            const mlp::Packed *Pg = P;
            asm volatile("" : "+s"(Pg));
            learned16(G, occupancy, hist + m0 * rowp, rowp, n16, cf_s + 16 * w, live_s + 16 * w, xs_all[w],
                      a1_all[w], Pg, est + h0 + m0);
            __syncthreads();
        }
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
