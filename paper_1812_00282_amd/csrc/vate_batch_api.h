// C ABI of the batched VATE path (declared in include/vate_batch.h).
// Included at the end of vate.hip, after the single-sketch entry points.

struct vate_batch {
    uint32_t S;
    vate_sketch *sk[kBatchMax];
    BatchItem host_items[kBatchMax];
    BatchItem *items;                    // device copy (caller-owned block)
    BatchTables *tab;                    // device tables (same block)
    const unsigned long long *n_pairs;   // device packet counts, one per sketch
    BatchTune tune;
    uint32_t cus;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int has_graph;
    int dead;
    char err[256];
};

static int bfail(vate_batch *b, int code, const char *msg)
{
    if (b) {
        snprintf(b->err, sizeof(b->err), "%s", msg);
        if (code == VATE_E_DEVICE) b->dead = 1;
    }
    return code;
}

static int bcheck(vate_batch *b, hipError_t e, const char *what)
{
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[200];
        snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
        return bfail(b, VATE_E_DEVICE, buf);
    }
    return VATE_OK;
}

static size_t batch_items_bytes(uint32_t n) { return align256(sizeof(BatchItem) * (size_t)n); }

static BatchTune default_tune(uint32_t cus)
{
    BatchTune t;
    t.ingest_tile = 8192;
    t.census_tile = 4096;
    t.estimate_block = 256;
    t.grid_preserve = cus;
    t.grid_ingest = 8 * cus;
    t.grid_census = 4 * cus;
    t.grid_estimate = 8 * cus;
    t.estimate_lanes = 1;
    t.census_unroll = 1;
    return t;
}

static void batch_phase(vate_batch *b, int ph, hipStream_t st)
{
    const BatchTune &t = b->tune;
    switch (ph) {
    case PH_PRESERVE: k_batch_preserve<<<t.grid_preserve, 256, 0, st>>>(b->items, b->S, b->tab); break;
    case PH_INGEST: k_batch_ingest<<<t.grid_ingest, 256, 0, st>>>(b->items, b->S, b->n_pairs, t, b->tab); break;
    case PH_CENSUS:
        if (t.census_unroll == 4) k_batch_census<4><<<t.grid_census, 256, 0, st>>>(b->items, b->S, t, b->tab);
        else if (t.census_unroll == 2) k_batch_census<2><<<t.grid_census, 256, 0, st>>>(b->items, b->S, t, b->tab);
        else k_batch_census<1><<<t.grid_census, 256, 0, st>>>(b->items, b->S, t, b->tab);
        break;
    default:
        if (t.estimate_lanes == 16)
            k_batch_estimate<16><<<t.grid_estimate, t.estimate_block, 0, st>>>(b->items, b->S, t, b->tab);
        else if (t.estimate_lanes == 4)
            k_batch_estimate<4><<<t.grid_estimate, t.estimate_block, 0, st>>>(b->items, b->S, t, b->tab);
        else
            k_batch_estimate<1><<<t.grid_estimate, t.estimate_block, 0, st>>>(b->items, b->S, t, b->tab);
        break;
    }
}

static void batch_enqueue(vate_batch *b, unsigned long long adv_mask, hipStream_t st)
{
    k_batch_begin<<<1, 64, 0, st>>>(b->items, b->S, b->n_pairs, adv_mask, b->tune, b->tab);
    for (int ph = 0; ph < PH_COUNT; ++ph) batch_phase(b, ph, st);
}

static bool batch_tune_valid(const BatchTune &t)
{
    return t.ingest_tile >= 512 && t.ingest_tile % 512 == 0 && t.census_tile >= 256 && t.census_tile % 256 == 0 &&
           (t.estimate_block == 64 || t.estimate_block == 128 || t.estimate_block == 256) && t.grid_preserve >= 1 &&
           t.grid_ingest >= 1 && t.grid_census >= 1 && t.grid_estimate >= 1 && t.grid_preserve <= 65536 &&
           t.grid_ingest <= 65536 && t.grid_census <= 65536 && t.grid_estimate <= 65536 &&
           (t.estimate_lanes == 1 || t.estimate_lanes == 4 || t.estimate_lanes == 16) &&
           (t.census_unroll == 1 || t.census_unroll == 2 || t.census_unroll == 4);
}

extern "C" {

int vate_batch_bytes(uint32_t n, size_t *bytes)
{
    if (!bytes || n < 1 || n > kBatchMax) return VATE_E_INVAL;
    *bytes = batch_items_bytes(n) + align256(sizeof(BatchTables));
    return VATE_OK;
}

int vate_batch_create(vate_sketch *const *sketches, uint32_t n, void *batch_dev, const uint64_t *n_pairs_dev,
                      vate_batch **out)
{
    if (!out) return VATE_E_INVAL;
    *out = nullptr;
    if (!sketches || n < 1 || n > kBatchMax || !batch_dev || !n_pairs_dev ||
        (reinterpret_cast<uintptr_t>(batch_dev) & 255u) || (reinterpret_cast<uintptr_t>(n_pairs_dev) & 7u))
        return VATE_E_INVAL;
    for (uint32_t i = 0; i < n; ++i) {
        if (!sketches[i] || sketches[i]->dead) return VATE_E_INVAL;
        for (uint32_t j = 0; j < i; ++j)
            if (sketches[j] == sketches[i]) return VATE_E_INVAL;
    }
    vate_batch *b = new (std::nothrow) vate_batch();
    if (!b) return VATE_E_NOMEM;
    b->S = n;
    b->items = static_cast<BatchItem *>(batch_dev);
    b->tab = reinterpret_cast<BatchTables *>(static_cast<uint8_t *>(batch_dev) + batch_items_bytes(n));
    b->n_pairs = reinterpret_cast<const unsigned long long *>(n_pairs_dev);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    b->cus = (uint32_t)cus;
    b->tune = default_tune(b->cus);
    for (uint32_t i = 0; i < n; ++i) {
        vate_sketch *s = sketches[i];
        b->sk[i] = s;
        BatchItem &it = b->host_items[i];
        memset(&it, 0, sizeof(it));
        it.G = s->G;
        it.pool = s->pool;
        it.st = s->st;
        it.bitmap = s->bitmap;
        const bool exact = s->p.width != 4 && s->p.width != 8 && s->p.width != 16;
        it.nchunks = exact ? s->G.N / 32 : s->pool_bytes / 16;   // groups of 32 counters / 16-byte chunks
        it.max_block_chunks = s->max_block_chunks;               // in the same units
        it.width = exact ? 0u : s->p.width;
        it.kprime = s->p.k;
    }
    hipError_t e = hipMemcpy(b->items, b->host_items, sizeof(BatchItem) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return VATE_E_DEVICE;
    }
    *out = b;
    return VATE_OK;
}

int vate_batch_set_io(vate_batch *b, uint32_t i, const uint32_t *pairs_dev, uint64_t pairs_capacity,
                      const uint32_t *hosts_dev, uint32_t n_hosts, uint32_t kprime, float *est_dev,
                      uint32_t *live_dev)
{
    if (!b) return VATE_E_INVAL;
    if (b->dead) return VATE_E_DEVICE;
    if (i >= b->S) return bfail(b, VATE_E_INVAL, "sketch index out of range");
    if ((reinterpret_cast<uintptr_t>(pairs_dev) & 15u) || (reinterpret_cast<uintptr_t>(hosts_dev) & 3u) ||
        (reinterpret_cast<uintptr_t>(est_dev) & 3u) || (reinterpret_cast<uintptr_t>(live_dev) & 3u))
        return bfail(b, VATE_E_INVAL, "pairs must be 16-byte, hosts/est/live 4-byte aligned");
    if (n_hosts > 0 && (!hosts_dev || !est_dev)) return bfail(b, VATE_E_INVAL, "hosts and est required");
    if (kprime < 1 || kprime > b->sk[i]->p.k) return bfail(b, VATE_E_INVAL, "k' must be in [1, k]");
    BatchItem &it = b->host_items[i];
    it.pairs = pairs_dev;
    it.pairs_cap = pairs_dev ? pairs_capacity : 0;
    it.hosts = hosts_dev;
    it.n_hosts = n_hosts;
    it.kprime = kprime;
    it.est = est_dev;
    it.live = live_dev;
    hipError_t e = hipMemcpy(b->items + i, &it, sizeof(BatchItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(b, VATE_E_DEVICE, hipGetErrorString(e));
    return VATE_OK;
}

int vate_batch_slice(vate_batch *b, void *stream)
{
    if (!b) return VATE_E_INVAL;
    if (b->dead) return VATE_E_DEVICE;
    unsigned long long mask = 0;
    for (uint32_t i = 0; i < b->S; ++i) {
        if (b->sk[i]->dead) return bfail(b, VATE_E_DEVICE, "a member sketch has a device error");
        if (b->sk[i]->closed) mask |= 1ull << i;
    }
    batch_enqueue(b, mask, static_cast<hipStream_t>(stream));
    int rc = bcheck(b, hipSuccess, "batch slice");
    if (rc != VATE_OK) return rc;
    for (uint32_t i = 0; i < b->S; ++i) b->sk[i]->closed = 1;
    return VATE_OK;
}

int vate_batch_capture(vate_batch *b, void *stream)
{
    if (!b) return VATE_E_INVAL;
    if (b->dead) return VATE_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!st) return bfail(b, VATE_E_INVAL, "capture needs a non-default stream");
    if (b->has_graph) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->has_graph = 0;
    }
    const unsigned long long all = b->S == 64 ? ~0ull : ((1ull << b->S) - 1ull);
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return bcheck(b, e, "begin capture");
    batch_enqueue(b, all, st);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return bcheck(b, e, "end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bcheck(b, e, "instantiate");
    }
    b->graph = g;
    b->exec = x;
    b->has_graph = 1;
    return VATE_OK;
}

int vate_batch_replay(vate_batch *b, void *stream)
{
    if (!b) return VATE_E_INVAL;
    if (b->dead) return VATE_E_DEVICE;
    if (!b->has_graph) return bfail(b, VATE_E_STATE, "no captured graph (call vate_batch_capture)");
    for (uint32_t i = 0; i < b->S; ++i)
        if (!b->sk[i]->closed) return bfail(b, VATE_E_STATE, "replay advances every sketch: all must be closed");
    int rc = bcheck(b, hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)), "graph launch");
    if (rc != VATE_OK) return rc;
    return VATE_OK;
}

int vate_batch_get_tune(const vate_batch *b, vate_batch_tune *t)
{
    if (!b || !t) return VATE_E_INVAL;
    t->ingest_tile = b->tune.ingest_tile;
    t->census_tile = b->tune.census_tile;
    t->estimate_block = b->tune.estimate_block;
    t->grid_preserve = b->tune.grid_preserve;
    t->grid_ingest = b->tune.grid_ingest;
    t->grid_census = b->tune.grid_census;
    t->grid_estimate = b->tune.grid_estimate;
    t->estimate_lanes = b->tune.estimate_lanes;
    t->census_unroll = b->tune.census_unroll;
    return VATE_OK;
}

int vate_batch_set_tune(vate_batch *b, const vate_batch_tune *t)
{
    if (!b || !t) return VATE_E_INVAL;
    BatchTune n;
    n.ingest_tile = t->ingest_tile;
    n.census_tile = t->census_tile;
    n.estimate_block = t->estimate_block;
    n.grid_preserve = t->grid_preserve;
    n.grid_ingest = t->grid_ingest;
    n.grid_census = t->grid_census;
    n.grid_estimate = t->grid_estimate;
    n.estimate_lanes = t->estimate_lanes;
    n.census_unroll = t->census_unroll;
    if (!batch_tune_valid(n)) return bfail(b, VATE_E_INVAL, "invalid tuning parameters");
    b->tune = n;
    return VATE_OK;
}

// Time each phase's candidate launch shapes on the batch's current slice
// (ingest, census and estimate are idempotent within a slice, so re-running
// them leaves the state as it was) and keep the fastest per phase.
int vate_batch_autotune(vate_batch *b, void *stream, char *report, size_t report_len)
{
    if (!b) return VATE_E_INVAL;
    if (b->dead) return VATE_E_DEVICE;
    for (uint32_t i = 0; i < b->S; ++i)
        if (!b->sk[i]->closed) return bfail(b, VATE_E_STATE, "autotune needs every sketch closed (run a slice)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(b, VATE_E_DEVICE, "event create");
    const uint32_t C = b->cus;
    BatchTune best = b->tune;
    std::string rep = "{\"candidates\":[";
    bool first = true;
    auto time_phase = [&](int ph, const BatchTune &cand, float *ms) -> int {
        b->tune = cand;
        float bestms = 1e30f;
        for (int r = 0; r < 3; ++r) {
            k_batch_begin<<<1, 64, 0, st>>>(b->items, b->S, b->n_pairs, 0ull, cand, b->tab);
            if (ph == PH_ESTIMATE || ph == PH_CENSUS) {
                // the census is cleared by begin; rebuild it before timing the estimate
                if (ph == PH_ESTIMATE) {
                    batch_phase(b, PH_CENSUS, st);
                    k_batch_reset_claim<<<1, 64, 0, st>>>(b->tab, PH_ESTIMATE);
                }
            }
            (void)hipEventRecord(e0, st);
            batch_phase(b, ph, st);
            (void)hipEventRecord(e1, st);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) return bcheck(b, e, "autotune");
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (t < bestms) bestms = t;
        }
        *ms = bestms;
        return VATE_OK;
    };
    const char *names[PH_COUNT] = {"preserve", "ingest", "census", "estimate"};
    float best_ms[PH_COUNT] = {0.f, 1e30f, 1e30f, 1e30f};
    // Per phase: tile size x a second axis x grid size (workgroups per CU).
    // The second axis is the census's chunks in flight per thread and the
    // estimate's lanes per host (how many lanes share one host's g gathers);
    // the ingest has none.
    const uint32_t tiles[3][3] = {{2048, 8192, 32768}, {1024, 4096, 16384}, {64, 128, 256}};
    const uint32_t axis[3][3] = {{0, 0, 0}, {1, 2, 4}, {1, 4, 16}};
    const uint32_t n_axis[3] = {1, 3, 3};
    const uint32_t grids[3][4] = {{2, 4, 8, 16}, {2, 4, 8, 16}, {4, 8, 16, 32}};
    for (int ph = PH_INGEST; ph <= PH_ESTIMATE; ++ph) {
        for (int ti = 0; ti < 3; ++ti)
            for (uint32_t ai = 0; ai < n_axis[ph - 1]; ++ai)
                for (int gi = 0; gi < 4; ++gi) {
                    BatchTune cand = best;
                    const uint32_t tv = tiles[ph - 1][ti], av = axis[ph - 1][ai], gv = grids[ph - 1][gi] * C;
                    if (ph == PH_INGEST) { cand.ingest_tile = tv; cand.grid_ingest = gv; }
                    if (ph == PH_CENSUS) { cand.census_tile = tv; cand.census_unroll = av; cand.grid_census = gv; }
                    if (ph == PH_ESTIMATE) { cand.estimate_block = tv; cand.estimate_lanes = av; cand.grid_estimate = gv; }
                    float ms = 0.f;
                    int rc = time_phase(ph, cand, &ms);
                    if (rc != VATE_OK) {
                        b->tune = best;
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                        return rc;
                    }
                    char buf[200];
                    snprintf(buf, sizeof(buf), "%s{\"phase\":\"%s\",\"tile\":%u,\"%s\":%u,\"grid\":%u,\"ms\":%.5f}",
                             first ? "" : ",", names[ph], tv, ph == PH_ESTIMATE ? "lanes" : "unroll", av, gv, ms);
                    first = false;
                    rep += buf;
                    if (ms < best_ms[ph]) {
                        best_ms[ph] = ms;
                        best = cand;
                    }
                }
        b->tune = best;
    }
    // leave the slice's outputs as a plain slice would: tables, census, estimate
    k_batch_begin<<<1, 64, 0, st>>>(b->items, b->S, b->n_pairs, 0ull, best, b->tab);
    batch_phase(b, PH_INGEST, st);
    batch_phase(b, PH_CENSUS, st);
    batch_phase(b, PH_ESTIMATE, st);
    hipError_t e = hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bcheck(b, e, "autotune");
    char buf[480];
    snprintf(buf, sizeof(buf),
             "],\"best\":{\"ingest_tile\":%u,\"grid_ingest\":%u,\"census_tile\":%u,\"census_unroll\":%u,"
             "\"grid_census\":%u,\"estimate_block\":%u,\"estimate_lanes\":%u,\"grid_estimate\":%u,"
             "\"ms\":{\"ingest\":%.5f,\"census\":%.5f,\"estimate\":%.5f}}}",
             best.ingest_tile, best.grid_ingest, best.census_tile, best.census_unroll, best.grid_census,
             best.estimate_block, best.estimate_lanes, best.grid_estimate, best_ms[PH_INGEST], best_ms[PH_CENSUS],
             best_ms[PH_ESTIMATE]);
    rep += buf;
    if (report && report_len) snprintf(report, report_len, "%s", rep.c_str());
    if (b->has_graph) {   // the captured graph holds the old launch shapes
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->has_graph = 0;
    }
    return VATE_OK;
}

const char *vate_batch_last_error(const vate_batch *b)
{
    return b ? b->err : "";
}

void vate_batch_destroy(vate_batch *b)
{
    if (!b) return;
    if (b->has_graph) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
    }
    delete b;
}

}  // extern "C"
