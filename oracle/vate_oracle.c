/*
 * VATE CPU oracle.  TEST INFRASTRUCTURE ONLY: it exists so that the tests,
 * the smoke check and the benchmark's CPU-baseline leg can check the HIP
 * path; no product code path may call, link or load it.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * Plain, slow, obviously-correct C.  One value per AT is kept in a uint16_t
 * array (the packed 4/8/16-bit container layout is only produced on request
 * by o_pack_pool).  Estimates are computed in double precision.
 *
 * It follows the paper (Xu, Ding, Hu: "VATE: a trade-off between memory and
 * preserving time for high accuracy cardinalities estimation under sliding
 * time window", arXiv 1812.00282) step by step:
 *   - AT value range [0, 2k], 2k = inactive           (Sec. 3, InitAT/SetAT)
 *   - CheckAT                                          (Algorithm 1)
 *   - PreserveAT, general form (dist >= k)             (Algorithm 2)
 *   - PreserveAT, fast form at ACT in {0, k}           (Algorithm 3, Cor. 1)
 *   - 2k AT blocks, BACT^i = (BACT^0 + i) mod 2k       (Eq. 6-8)
 *   - block partition a = 2^c/(2k-1), remainder b      (Eq. 9-10, Fig. 4)
 *     or the low-deviation partition                   (Sec. 4.1, Fig. 5)
 *   - VAT_aip^i = ATP[H(aip,i)], bip sets VAT BH(bip)  (Sec. 4.1)
 *   - estimate g ln Z_p - g ln Z_v                     (Eq. 11, sign read as
 *     in Eq. 1 so that a host with traffic gets a positive estimate)
 *   - per-slice loop: scan pairs, estimate, BACT^0++, t++, preserve the two
 *     blocks whose ACT is 0 or k                        (Algorithm 4)
 *
 * Readings where the paper is silent or inconsistent:
 *   - H and BH are unspecified: mix = MurmurHash3's 32-bit finalizer fmix32;
 *     BH(bip) = floor(mix(bip ^ seed_b) * g / 2^32) (multiply-high range
 *     reduction); H(aip,i) = top c bits of mix(mix(aip ^ seed_a) ^ i*PHI).
 *   - Algorithm 4's block size 2^c/k conflicts with Eq. 9; Eq. 9 is used,
 *     with the block index clamped to 2k-1 (Fig. 4 puts the remainder there).
 *   - Algorithm 4 calls SetAT inside the maintenance loop; read as PreserveAT.
 *   - SetAT stores the AT's current ACT (Sec. 3), not 0.
 *   - Saturation (u_v = 0 or u_p = 0) is silent in the paper: the count is
 *     taken as 1 so the logarithm stays finite.
 *
 * Call sequence (mirrors the C-ABI): ingest* -> close -> estimate* ; the next
 * ingest or close first advances the clock and preserves (Algorithm 4 puts
 * estimation before BACT^0++ / t++ / preservation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHI 0x9E3779B9u

typedef struct {
    uint32_t c, w, k, g, partition;
    uint32_t counter;      /* 0: asynchronous timestamps (VATE); 1: distance
                              recorders (VDRE, the paper's baseline) */
    uint32_t blog;         /* 0: H as read from Sec. 4.1 (independent VATs);
                              b > 0: locality-blocked H, blocks of 2^b VATs */
    uint32_t seed_a, seed_b;
    uint64_t N;            /* 2^c ATs in the pool ATP */
    uint16_t *ATP;         /* AT values in [0, 2k] */
    uint64_t *blk_start;   /* 2k+1 entries: B[i] = [blk_start[i], blk_start[i+1]) */
    uint32_t BACT0;        /* ACT of block 0 (Eq. 7) */
    uint64_t t;            /* current time slice */
    int closed;            /* 1 once slice t has ended (estimates allowed) */
} o_vate;

/* ---- hashing (reading of Sec. 4.1's H and BH) ---- */

/* MurmurHash3 32-bit finalizer (Appleby), from its published description. */
uint32_t o_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

uint32_t o_hash_BH(uint32_t g, uint32_t seed_b, uint32_t bip)
{
    uint64_t m = o_fmix32(bip ^ seed_b);
    return (uint32_t)((m * (uint64_t)g) >> 32);
}

uint32_t o_hash_H(uint32_t c, uint32_t seed_a, uint32_t aip, uint32_t i)
{
    uint32_t x = o_fmix32(o_fmix32(aip ^ seed_a) ^ (uint32_t)(i * PHI));
    /* floor(x * 2^c / 2^32) */
    return (uint32_t)(((uint64_t)x << c) >> 32);
}

/* Locality-blocked H (an opt-in variant, not the paper's): VAT i of a host is
 * slot i mod 2^b of the host's block floor(i / 2^b), and that block sits at a
 * block-aligned position given by the top c - b bits of the same mix applied
 * to the block number.  b = 0 is o_hash_H. */
uint32_t o_hash_H_blocked(uint32_t c, uint32_t b, uint32_t seed_a, uint32_t aip, uint32_t i)
{
    if (b == 0)
        return o_hash_H(c, seed_a, aip, i);
    uint32_t j = i >> b;
    uint32_t x = o_fmix32(o_fmix32(aip ^ seed_a) ^ (uint32_t)(j * PHI));
    uint32_t block = (uint32_t)(((uint64_t)x << (c - b)) >> 32);   /* floor(x * 2^(c-b) / 2^32) */
    return (block << b) | (i & ((1u << b) - 1u));
}

uint32_t o_BH(const o_vate *s, uint32_t bip)
{
    return o_hash_BH(s->g, s->seed_b, bip);
}

uint32_t o_H(const o_vate *s, uint32_t aip, uint32_t i)
{
    return o_hash_H_blocked(s->c, s->blog, s->seed_a, aip, i);
}

/* ---- AT blocks (Eq. 6-10, Fig. 4 / Fig. 5) ---- */

uint32_t o_block_of(const o_vate *s, uint64_t pid)
{
    uint64_t twok = 2ull * s->k;
    if (s->partition == 0) {
        /* Fig. 4: the first 2k-1 blocks hold a ATs, the last holds b. */
        uint64_t a = s->N / (twok - 1);
        uint64_t bid = pid / a;
        return (uint32_t)(bid < twok - 1 ? bid : twok - 1);
    } else {
        /* Fig. 5: first 2k-b' blocks hold a', the last b' hold a'+1. */
        uint64_t ap = s->N / twok, bp = s->N % twok;
        if (pid < ap * (twok - bp))
            return (uint32_t)(pid / ap);
        return (uint32_t)((pid + twok - bp) / (ap + 1));
    }
}

/* BACT_t^i = (BACT_t^0 + i) mod 2k  (Eq. 8) */
uint32_t o_block_act(const o_vate *s, uint32_t i)
{
    return (s->BACT0 + i) % (2u * s->k);
}

uint32_t o_act_of(const o_vate *s, uint64_t pid)
{
    return o_block_act(s, o_block_of(s, pid));
}

/* ---- the four AT operations (Sec. 3) ---- */

/* Algorithm 1: active in W(t-k'+1, k') at the end of slice t. */
int o_checkAT(uint32_t value, uint32_t act, uint32_t k, uint32_t kprime)
{
    if (value == 2 * k)
        return 0;
    uint32_t dis = (act + 2 * k - value) % (2 * k);
    return dis <= kprime - 1;
}

/* Algorithm 2: general PreserveAT (mark inactive once dist >= k). */
uint32_t o_preserve_general(uint32_t value, uint32_t act, uint32_t k)
{
    uint32_t dis = (act + 2 * k - value) % (2 * k);
    if (dis >= k)
        return 2 * k;
    return value;
}

/* Algorithm 3: fast PreserveAT, only ever applied when ACT is 0 or k. */
uint32_t o_preserve_fast(uint32_t value, uint32_t act, uint32_t k)
{
    if (act == 0) {
        if (value <= k)              /* 0 <= Value <= k */
            return 2 * k;
    }
    if (act == k) {
        if (value >= k && value <= 2 * k - 1)
            return 2 * k;
        if (value == 0)
            return 2 * k;
    }
    return value;
}

/* ---- sketch lifecycle ---- */

o_vate *o_create(uint32_t c, uint32_t w, uint32_t k, uint32_t g,
                 uint32_t seed_a, uint32_t seed_b, uint32_t partition, uint32_t counter, uint32_t blog)
{
    if (c < 1 || c > 32 || k < 1 || g < 1 || counter > 1 || blog > 10 || blog > c)
        return NULL;
    if (w < 1 || w > 16)
        return NULL;
    if (w != 4 && w != 8 && w != 16 && c < 5)   /* exact packing: whole 32-bit words */
        return NULL;
    if (counter == 0 && (1ull << w) < 2ull * k + 1)   /* AT: ceil(log2(2k+1)) bits */
        return NULL;
    if (counter == 1 && (1ull << w) < 1ull * k + 1)   /* DR: ceil(log2(k+1)) bits */
        return NULL;
    if ((1ull << c) < 2ull * k)
        return NULL;
    o_vate *s = (o_vate *)calloc(1, sizeof(o_vate));
    if (!s)
        return NULL;
    s->c = c; s->w = w; s->k = k; s->g = g; s->partition = partition;
    s->counter = counter;
    s->blog = blog;
    s->seed_a = seed_a; s->seed_b = seed_b;
    s->N = 1ull << c;
    s->ATP = (uint16_t *)malloc(s->N * sizeof(uint16_t));
    s->blk_start = (uint64_t *)calloc(2ull * k + 1, sizeof(uint64_t));
    if (!s->ATP || !s->blk_start) {
        free(s->ATP); free(s->blk_start); free(s);
        return NULL;
    }
    /* InitAT on every AT of ATP (Algorithm 4 init): value 2k.  A DR starts
     * as "not seen within k slices": value k. */
    for (uint64_t p = 0; p < s->N; p++)
        s->ATP[p] = (uint16_t)(counter == 0 ? 2 * k : k);
    /* Block ranges found by scanning block_of over the pool: block i starts
     * at the first pid mapped to it (empty blocks start where the next does). */
    for (uint64_t i = 0; i <= 2ull * k; i++)
        s->blk_start[i] = s->N;
    for (uint64_t p = s->N; p-- > 0;)
        s->blk_start[o_block_of(s, p)] = p;
    for (uint64_t i = 2ull * k; i-- > 0;)
        if (s->blk_start[i] > s->blk_start[i + 1])
            s->blk_start[i] = s->blk_start[i + 1];
    s->BACT0 = 0;
    s->t = 0;
    s->closed = 0;
    return s;
}

void o_destroy(o_vate *s)
{
    if (!s)
        return;
    free(s->ATP);
    free(s->blk_start);
    free(s);
}

/* End of Algorithm 4's loop body: BACT^0++, t++, then PreserveAT over every
 * block whose ACT became 0 or k. */
static void o_advance(o_vate *s)
{
    s->BACT0 = (s->BACT0 + 1) % (2 * s->k);
    s->t = s->t + 1;
    if (s->counter == 1) {
        /* DR (Sec. 1): every counter grows by one when the window slides;
         * it saturates at k, which already means inactive for every k' <= k. */
        for (uint64_t p = 0; p < s->N; p++)
            if (s->ATP[p] < s->k)
                s->ATP[p] = (uint16_t)(s->ATP[p] + 1);
        s->closed = 0;
        return;
    }
    for (uint32_t i = 0; i < 2 * s->k; i++) {
        uint32_t bact = o_block_act(s, i);
        if (bact == 0 || bact == s->k) {
            for (uint64_t p = s->blk_start[i]; p < s->blk_start[i + 1]; p++)
                s->ATP[p] = (uint16_t)o_preserve_fast(s->ATP[p], bact, s->k);
        }
    }
    s->closed = 0;
}

/* Scan IP pairs of the current slice (Algorithm 4 scan loop).  pairs holds n
 * interleaved (aip, bip) uint32 values. */
void o_ingest(o_vate *s, const uint32_t *pairs, uint64_t n)
{
    if (s->closed)
        o_advance(s);
    for (uint64_t j = 0; j < n; j++) {
        uint32_t aip = pairs[2 * j], bip = pairs[2 * j + 1];
        uint32_t vid = o_BH(s, bip);
        uint32_t pid = o_H(s, aip, vid);
        if (s->counter == 1) {
            s->ATP[pid] = 0;                      /* a DR is reset to 0 */
            continue;
        }
        uint32_t bid = o_block_of(s, pid);
        uint32_t act = (s->BACT0 + bid) % (2 * s->k);
        s->ATP[pid] = (uint16_t)act;              /* SetAT */
    }
}

/* pid = H(aip, BH(bip)) of each pair (the AT a packet sets). */
void o_packet_pids(const o_vate *s, const uint32_t *pairs, uint64_t n,
                   uint32_t *pids)
{
    for (uint64_t j = 0; j < n; j++)
        pids[j] = o_H(s, pairs[2 * j], o_BH(s, pairs[2 * j + 1]));
}

/* End the current slice (an empty slice if nothing was ingested). */
void o_close(o_vate *s)
{
    if (s->closed)
        o_advance(s);
    s->closed = 1;
}

/* DR check (Sec. 1): active in W(t-k'+1, k') iff its value is below k'. */
int o_checkDR(uint32_t value, uint32_t kprime)
{
    return value < kprime;
}

/* CheckAT or the DR check of pool slot pid. */
static int o_check(const o_vate *s, uint64_t pid, uint32_t kprime)
{
    if (s->counter == 1)
        return o_checkDR(s->ATP[pid], kprime);
    return o_checkAT(s->ATP[pid], o_act_of(s, pid), s->k, kprime);
}

/* Census of the pool at the end of the slice: hist[d] for d < k counts ATs
 * whose value is not 2k and whose distance is d; hist[k] counts the rest.
 * For DR counters the distance is the value itself. */
void o_census(const o_vate *s, uint64_t *hist)
{
    for (uint32_t d = 0; d <= s->k; d++)
        hist[d] = 0;
    for (uint64_t p = 0; p < s->N; p++) {
        uint32_t v = s->ATP[p];
        if (s->counter == 1) {
            hist[v < s->k ? v : s->k]++;
            continue;
        }
        uint32_t act = o_act_of(s, p);
        if (v == 2 * s->k) {
            hist[s->k]++;
            continue;
        }
        uint32_t dis = (act + 2 * s->k - v) % (2 * s->k);   /* Eq. 5 */
        hist[dis < s->k ? dis : s->k]++;
    }
}

/* Number of inactive ATs in the pool for window k' (numerator of Z_p). */
uint64_t o_pool_inactive(const o_vate *s, uint32_t kprime)
{
    uint64_t u = 0;
    for (uint64_t p = 0; p < s->N; p++)
        if (!o_check(s, p, kprime))
            u++;
    return u;
}

/* Eq. 11 with the sign of Eq. 1: n = g ln Z_p - g ln Z_v, in double. */
double o_estimate_counts(uint64_t u_v, uint64_t u_p, uint32_t g, uint64_t N)
{
    if (u_v == 0)
        u_v = 1;
    if (u_p == 0)
        u_p = 1;
    double Zv = (double)u_v / (double)g;
    double Zp = (double)u_p / (double)N;
    return (double)g * log(Zp) - (double)g * log(Zv);
}

/* Estimate every host in hosts[0..nh) for window k' at the end of the slice
 * (Algorithm 4 estimation loop).  est must hold nh doubles; live (nullable)
 * gets the number of active VATs; hist (nullable) nh*(k+1) entries of the
 * host's VAT distance histogram, same binning as o_census.  Returns 0, or -1
 * if the slice is not closed or k' is out of range. */
int o_estimate(const o_vate *s, const uint32_t *hosts, uint64_t nh,
               uint32_t kprime, double *est, uint32_t *live, uint32_t *hist)
{
    if (!s->closed || kprime < 1 || kprime > s->k)
        return -1;
    uint64_t u_p = o_pool_inactive(s, kprime);
    for (uint64_t h = 0; h < nh; h++) {
        uint32_t aip = hosts[h];
        uint64_t u_v = 0;
        if (hist)
            for (uint32_t d = 0; d <= s->k; d++)
                hist[h * (s->k + 1) + d] = 0;
        for (uint32_t i = 0; i < s->g; i++) {
            uint32_t pid = o_H(s, aip, i);             /* VAT_aip^i */
            uint32_t v = s->ATP[pid];
            if (!o_check(s, pid, kprime))
                u_v++;
            if (hist && s->counter == 1) {
                hist[h * (s->k + 1) + (v < s->k ? v : s->k)]++;
                continue;
            }
            uint32_t act = o_act_of(s, pid);
            if (hist) {
                uint32_t bin = s->k;
                if (v != 2 * s->k) {
                    uint32_t dis = (act + 2 * s->k - v) % (2 * s->k);
                    if (dis < s->k)
                        bin = dis;
                }
                hist[h * (s->k + 1) + bin]++;
            }
        }
        if (live)
            live[h] = (uint32_t)(s->g - u_v);
        est[h] = o_estimate_counts(u_v, u_p, s->g, s->N);
    }
    return 0;
}

/* ---- state access ---- */

uint64_t o_N(const o_vate *s) { return s->N; }
uint64_t o_t(const o_vate *s) { return s->t; }
uint32_t o_bact0(const o_vate *s) { return s->BACT0; }
int o_closed(const o_vate *s) { return s->closed; }
uint64_t o_blk_start(const o_vate *s, uint32_t i) { return s->blk_start[i]; }

void o_values(const o_vate *s, uint16_t *out)
{
    memcpy(out, s->ATP, s->N * sizeof(uint16_t));
}

void o_set_values(o_vate *s, const uint16_t *in, uint64_t t, uint32_t bact0,
                  int closed)
{
    memcpy(s->ATP, in, s->N * sizeof(uint16_t));
    s->t = t;
    s->BACT0 = bact0;
    s->closed = closed;
}

/* Pool in the packed layout: AT p occupies bits [p*w, p*w+w) of a
 * little-endian bit string (w=4: low nibble = even p; w=8: byte p; w=16: LE
 * uint16; any other w: counters back to back).  out holds N*w/8 bytes. */
void o_pack_pool(const o_vate *s, uint8_t *out)
{
    if (s->w != 4 && s->w != 8 && s->w != 16) {
        memset(out, 0, (size_t)(s->N * s->w / 8));
        for (uint64_t p = 0; p < s->N; p++)
            for (uint32_t j = 0; j < s->w; j++)
                if ((s->ATP[p] >> j) & 1u) {
                    const uint64_t bit = p * s->w + j;
                    out[bit >> 3] |= (uint8_t)(1u << (bit & 7));
                }
        return;
    }
    if (s->w == 8) {
        for (uint64_t p = 0; p < s->N; p++)
            out[p] = (uint8_t)s->ATP[p];
    } else if (s->w == 16) {
        for (uint64_t p = 0; p < s->N; p++) {
            out[2 * p] = (uint8_t)(s->ATP[p] & 0xff);
            out[2 * p + 1] = (uint8_t)(s->ATP[p] >> 8);
        }
    } else {
        for (uint64_t p = 0; p < s->N; p += 2)
            out[p / 2] = (uint8_t)((s->ATP[p] & 0xf) | ((s->ATP[p + 1] & 0xf) << 4));
    }
}
