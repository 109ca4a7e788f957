/*
 * vate.h - C ABI of the MI355X (gfx950) VATE library, libvate.so.
 *
 * VATE (Xu, Ding, Hu, arXiv 1812.00282) estimates, at the end of every time
 * slice, the number of distinct opposite hosts (bip) each ANet host (aip)
 * talked to in the last k' <= k slices.  All hosts share one pool ATP of 2^c
 * asynchronous timestamps (ATs); host aip owns g virtual ATs
 * VAT_aip^i = ATP[H(aip, i)], and a packet <aip, bip> sets VAT_aip^BH(bip)
 * (Sec. 4.1).  An AT holds its block's ACT from the slice it was last set, or
 * 2k when inactive (Sec. 3); the pool is cut into 2k blocks with staggered
 * ACTs (Eq. 6-10) so only two blocks need maintenance per slice (Alg. 4).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (hipMalloc / torch CUDA
 *    memory) owned by the caller, which keeps them alive until the work
 *    enqueued on `stream` has finished (and pool/state until vate_destroy).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously on it; only argument validation is synchronous
 *    unless stated otherwise.
 *  - The library owns only the small host-side vate_sketch handle.
 *  - Every call returns a status code (VATE_OK = 0).  No C++ exception
 *    crosses the ABI.  A HIP error is sticky: it is recorded on the handle,
 *    every later call returns VATE_E_DEVICE, and vate_last_error() gives text.
 *  - Calls on one sketch must not run concurrently from several host threads.
 *
 * Hash functions (H and BH are left unspecified by Sec. 4.1; this library
 * fixes them, with mix = MurmurHash3's 32-bit finalizer fmix32):
 *    BH(bip)   = floor(mix(bip ^ seed_b) * g / 2^32)                 in [0, g)
 *    H(aip, i) = floor(mix(mix(aip ^ seed_a) ^ (i * 0x9E3779B9)) * 2^c / 2^32)
 *
 * Pool layout in HBM: AT p occupies bits [p*width, (p+1)*width) of the pool
 * byte array, little-endian (width 4: even p in the low nibble of byte p/2;
 * width 16: little-endian uint16 p; any other width: counters packed back to
 * back in little-endian 32-bit words, so 32 counters fill exactly `width`
 * words - the paper's exact-width pool, Sec. 3 and Sec. 5).  Pool bytes =
 * 2^c * width / 8.
 */
#ifndef VATE_H
#define VATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define VATE_OK            0
#define VATE_E_INVAL       1  /* bad parameter, pointer, size or alignment */
#define VATE_E_STATE       2  /* call not allowed in the current slice phase */
#define VATE_E_DEVICE      3  /* HIP error (sticky on the handle) */
#define VATE_E_NOMEM       4  /* host allocation failed */
#define VATE_E_UNSUPPORTED 5  /* valid request outside this build's limits */

/* Sketch parameters (Alg. 4 inputs c, k, k'; g of Sec. 4.1). */
typedef struct vate_params {
    uint32_t log2_pool;  /* c: the pool holds N = 2^c ATs; 1 <= c <= 32 and
                            N >= 2k; widths 4/8/16 need N*width/8 >= 16 bytes,
                            other widths N >= 32 */
    uint32_t width;      /* bits per AT, 1..16; the AT needs ceil(log2(2k+1))
                            bits (Sec. 3), so 2^width >= 2k+1.  4, 8 and 16 use
                            nibble/byte/short containers; any other width packs
                            the ATs exactly (e.g. 7 bits at k = 60, 10 at
                            k = 300), in the single-sketch and batched calls */
    uint32_t k;          /* longest window, in slices (Sec. 1); k >= 1 */
    uint32_t g;          /* VATs per host (Sec. 4.1); 1 <= g <= 65535 */
    uint32_t partition;  /* 0: Eq. 9-10 blocks (Fig. 4: 2k-1 blocks of
                            floor(N/(2k-1)) ATs, the remainder in the last);
                            1: low-deviation blocks (Fig. 5) */
    uint32_t seed_a;     /* seed of H */
    uint32_t seed_b;     /* seed of BH */
    uint32_t counter;    /* 0: asynchronous timestamps (VATE, Sec. 3);
                            1: distance recorders (VDRE, the baseline of Sec. 5:
                            a DR holds the slices since its last hit, saturating
                            at k, is reset to 0 by a packet and incremented for
                            the whole pool at every slide, Sec. 1; it needs
                            2^width >= k+1).  Same hashing, estimates and ABI. */
    uint32_t block_log2; /* 0: H as above (the paper's independent VATs).
                            b in 1..10, b <= c: locality-blocked H, not the
                            paper's - VAT i of a host is slot i mod 2^b of the
                            host's block floor(i / 2^b), a run of 2^b
                            consecutive ATs whose position is the top c - b
                            bits of mix(mix(aip ^ seed_a) ^ floor(i/2^b) *
                            0x9E3779B9), times 2^b.  Same ABI; fewer cache
                            lines per host at a cost in estimator variance. */
} vate_params;

typedef struct vate_sketch vate_sketch;

/* Device memory a sketch needs: the pool (N*width/8 bytes, 256-byte aligned)
 * and a state block (clock t, BACT^0, flags, pool census, the activity
 * bitmap of N bits, 16 partial censuses of k counters; 256-byte aligned).
 * Validates *p.  Returns VATE_OK or VATE_E_INVAL. */
int vate_state_bytes(const vate_params *p, size_t *pool_bytes, size_t *state_bytes);

/* Create a sketch over caller-owned pool_dev / state_dev (sizes from
 * vate_state_bytes) and enqueue Alg. 4's initialisation on `stream`: InitAT
 * on every AT (value 2k), BACT^0 = 0, t = 0 (Alg. 4 init, Sec. 4.2 first
 * paragraph).  Slice 0 is then open for packets.  On success *out receives
 * the handle (free with vate_destroy).  Errors: VATE_E_INVAL (parameters,
 * NULL or misaligned pointers), VATE_E_NOMEM, VATE_E_DEVICE. */
int vate_create(const vate_params *p, void *pool_dev, void *state_dev,
                void *stream, vate_sketch **out);

/* Scan n IP pairs of the current slice (Alg. 4 scan loop; Sec. 4.2 "scanning
 * IP address pairs"): for each pair vid = BH(bip), pid = H(aip, vid), and
 * SetAT(ATP[pid]) stores the ACT of pid's block, (BACT^0 + block) mod 2k
 * (Eq. 8).  pairs_dev holds 2n uint32 values, interleaved aip, bip (8 bytes
 * per packet as in Sec. 4.2), 8-byte aligned.  n may be 0.  Any number of
 * calls per slice; order and duplicates within a slice do not matter
 * (Sec. 4.2's write-conflict argument).  If the previous slice was closed,
 * this first advances the clock and preserves (see vate_close_slice).
 * Errors: VATE_E_INVAL (NULL/misaligned pairs with n > 0), VATE_E_DEVICE. */
int vate_ingest(vate_sketch *s, const uint32_t *pairs_dev, size_t n, void *stream);

/* End the current slice: enqueue the pool census (the distance histogram of
 * every AT; Z_p of Eq. 11 for any k' follows from it).  Estimates for this
 * slice are allowed afterwards.  If the sketch was already closed, the clock
 * first advances through an empty slice.  Advancing is Alg. 4's end of loop:
 * BACT^0 = (BACT^0 + 1) mod 2k, t = t + 1, then PreserveAT (Alg. 3) on the
 * two blocks whose ACT became 0 or k (Cor. 1).  Errors: VATE_E_DEVICE. */
int vate_close_slice(vate_sketch *s, void *stream);

/* Estimate the cardinality of n_hosts hosts over W(t-k'+1, k') at the end of
 * the closed slice t (Alg. 4 estimation loop, Eq. 11; Sec. 4.2 "estimating
 * cardinality"):  est = g ln Z_p - g ln Z_v, where Z_v is the fraction of
 * the host's g VATs and Z_p the fraction of the pool that CheckAT (Alg. 1)
 * finds inactive for k'.  (Eq. 11 prints the opposite sign; Eq. 1's sign is
 * used so that a host with traffic gets a positive estimate.)  A count of
 * zero inactive ATs is taken as one.  Computed in FP32 from exact integer
 * counts: with D = u_p*g - N*u_v, x = D/(N*u_v), est = g*log1p(x) for
 * x >= -1/2, else g*log(u_p*g/(N*u_v)).
 *   hosts_dev: n_hosts uint32 aips.  est_dev: n_hosts float.
 *   live_dev (nullable): n_hosts uint32, number of active VATs for k'.
 *   hist_dev (nullable): n_hosts*(k+1) uint32, row-major; entry d < k counts
 *     the host's VATs whose value is not 2k and whose distance (Eq. 5) is d;
 *     entry k counts the rest.  Requires k <= 256.
 * Errors: VATE_E_STATE (slice not closed), VATE_E_INVAL (k' outside [1, k],
 * NULL/misaligned buffers), VATE_E_UNSUPPORTED (hist with k > 256),
 * VATE_E_DEVICE. */
int vate_estimate(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                  uint32_t kprime, float *est_dev, uint32_t *live_dev,
                  uint32_t *hist_dev, void *stream);

/* Device workspace (bytes) that vate_estimate_ws needs for n_hosts hosts:
 * about 8*g bytes per host (a 32-bit entry and a 32-bit slot for its live
 * copy per VAT, runs padded to 4) plus the run table.  Errors: VATE_E_INVAL. */
int vate_estimate_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes);

/* Same results as vate_estimate (same outputs, layouts, errors; any k for the
 * histogram), computed with the VAT lookups (Alg. 4's estimate loop, Alg. 1)
 * reordered for locality: the hosts' VATs are hashed once and sorted into
 * the workspace by pool slice of 2^20 ATs, each slice's lookups are tested
 * against that slice's activity bits for window k (held in LDS), only the
 * live VATs are kept and read from the pool for their distance, and every
 * host's distance histogram is rebuilt from them.  workspace_dev (256-byte
 * aligned, at least vate_estimate_workspace_bytes) is scratch owned by the
 * caller; calls that share a workspace must not overlap.  Sketches outside
 * the path's limits (g above the sort's capacity, the locality-blocked H)
 * fall back to vate_estimate's gather.  Errors: as vate_estimate, plus
 * VATE_E_INVAL for a missing or small workspace. */
int vate_estimate_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                     uint32_t kprime, float *est_dev, uint32_t *live_dev, uint32_t *hist_dev,
                     void *workspace_dev, size_t workspace_bytes, void *stream);

/* vate_estimate_ws for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the workspace is a fixed array of VATE_NOALLOC_SCRATCH_BYTES
 * in device memory that the library holds on every GPU it runs on, from
 * module load until the process ends.  No call allocates or frees anything.
 * Same arguments (minus the workspace), outputs, layouts and results as
 * vate_estimate_ws.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (from any
 * sketch, stream or host thread) race and must not be issued.  The host
 * count is limited by the array: at g = 1024 on a 2^28 pool about 7,900 hosts.
 * Errors: as vate_estimate_ws; VATE_E_INVAL when the host count needs more
 * workspace than VATE_NOALLOC_SCRATCH_BYTES (vate_estimate_workspace_bytes
 * tells); VATE_E_DEVICE if the array's device address cannot be found. */
#define VATE_NOALLOC_SCRATCH_BYTES (64u << 20)
int vate_estimate_noalloc(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                          uint32_t kprime, float *est_dev, uint32_t *live_dev,
                          uint32_t *hist_dev, void *stream);

/* vate_estimate_ws in two parts, for a host list that stays the same from
 * slice to slice (the monitored hosts of Alg. 4's ANet): the VAT addresses
 * depend only on the hosts and H, not on the pool, so
 *   vate_estimate_plan hashes and sorts the hosts' VATs into the workspace
 *     (any slice phase; hosts_dev is read during the call's stream work only),
 *   vate_estimate_run answers a closed slice from that plan (lookups and
 *     histograms only) with vate_estimate_ws's outputs and layouts.
 * The plan belongs to the sketch and to this workspace and host count; it
 * stays valid until the workspace is used by another estimate call.  A
 * changed host list needs a new plan.  Errors: VATE_E_UNSUPPORTED (plan for a
 * sketch outside the partitioned path), VATE_E_STATE (run without a plan for
 * this workspace and n_hosts, or slice not closed), VATE_E_INVAL, VATE_E_DEVICE. */
int vate_estimate_plan(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                       void *workspace_dev, size_t workspace_bytes, void *stream);
int vate_estimate_run(vate_sketch *s, size_t n_hosts, uint32_t kprime, float *est_dev,
                      uint32_t *live_dev, uint32_t *hist_dev, void *workspace_dev,
                      size_t workspace_bytes, void *stream);

/* Estimates for several windows k'_1 < ... < k'_m (m <= 64, each in [1, k],
 * given in host memory) from one pass over each host's VATs: any window up
 * to k is answerable from the same state (Sec. 3, CheckAT; Sec. 4.1).
 * est_dev receives n_hosts*m floats, row-major [host][window].  Lookups as in
 * vate_estimate_ws; workspace from vate_estimate_multi_workspace_bytes.
 * Errors: as vate_estimate_ws; VATE_E_INVAL for bad window lists. */
int vate_estimate_multi_workspace_bytes(const vate_sketch *s, size_t n_hosts, size_t *bytes);
int vate_estimate_multi_ws(vate_sketch *s, const uint32_t *hosts_dev, size_t n_hosts,
                           const uint32_t *kprimes, uint32_t m, float *est_dev,
                           void *workspace_dev, size_t workspace_bytes, void *stream);

/* Pool census of the closed slice, copied to host memory: census_host[d] for
 * d < k counts ATs whose value is not 2k with distance d; census_host[k]
 * counts the rest (inactive for every k').  Synchronises `stream`.
 * Errors: VATE_E_STATE (not closed), VATE_E_INVAL, VATE_E_DEVICE. */
int vate_read_census(vate_sketch *s, uint64_t *census_host, void *stream);

/* Checkpoint: synchronise `stream`, copy the pool (pool_bytes bytes) to
 * pool_dst (host or device memory; NULL skips the copy) and return the clock
 * t, BACT^0 and whether the slice is closed (1) or open (0).  The full VATE
 * state is (ATP, t, BACT^0) plus the parameters (Alg. 4).
 * Errors: VATE_E_INVAL, VATE_E_DEVICE. */
int vate_read_state(vate_sketch *s, void *pool_dst, uint64_t *t, uint32_t *bact0,
                    int *closed, void *stream);

/* Restore a checkpoint taken with vate_read_state from a sketch with the same
 * parameters: copy pool_src (host or device, pool_bytes bytes) into the pool,
 * set t and BACT^0 (bact0 < 2k) and the phase; a closed phase recomputes the
 * census.  Enqueued on `stream`; pool_src must stay valid until it has run.
 * Errors: VATE_E_INVAL, VATE_E_DEVICE. */
int vate_load_state(vate_sketch *s, const void *pool_src, uint64_t t, uint32_t bact0,
                    int closed, void *stream);

/* Text of the last error on the handle ("" if none); never NULL. */
const char *vate_last_error(const vate_sketch *s);

/* Static description of a status code. */
const char *vate_status_string(int code);

/* Release the host handle (device memory stays the caller's).  NULL is a
 * no-op.  Does not synchronise; the caller must not free pool/state while
 * enqueued work still uses them. */
void vate_destroy(vate_sketch *s);

/* Host-side evaluation of the library's own hash and block functions, the
 * same inline code the kernels run, for host-side tests.
 * vate_host_hash: which = 0 gives BH(x), 1 gives H(x, i).  vate_host_block:
 * block index of pid under *p (Eq. 9-10 or Fig. 5).  Return 0xFFFFFFFF for
 * invalid parameters. */
uint32_t vate_host_hash(const vate_params *p, uint32_t which, uint32_t x, uint32_t i);
uint32_t vate_host_block(const vate_params *p, uint64_t pid);

#ifdef __cplusplus
}
#endif

#endif /* VATE_H */
