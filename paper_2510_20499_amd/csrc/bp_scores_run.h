// bp_scores_run.h -- host side of bp_scores and bp_probe_order (included by
// bp_engine.hip after the kernels of bp_scores.h).
#pragma once

// Per-call work of the scores: packed bounds, row activities (slacks),
// partial sums of the chunks of the long rows, and a NaN flag.
struct ScWork {
    double2 *bnd;
    double2 *act;
    Acc *part;
    int32_t *flag;
};

// Bytes of each part of ScWork for an instance (each a multiple of 256).
struct ScWorkSize {
    size_t flag, bnd, act, part;
    size_t total() const { return flag + bnd + act + part; }
};

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

static ScWorkSize sc_work_size(const bp_instance *h) {
    ScWorkSize z;
    z.flag = 256;
    z.bnd = round256((size_t)std::max<int32_t>(h->n, 1) * sizeof(double2));
    z.act = round256((size_t)std::max<int32_t>(h->m, 1) * sizeof(double2));
    z.part = round256((size_t)std::max<int64_t>(h->sc_nchunks, 1) * 2 * sizeof(Acc));
    return z;
}

// ScWork carved out of one block of device memory of sc_work_size bytes.
static ScWork sc_work_at(const bp_instance *h, void *base) {
    const ScWorkSize z = sc_work_size(h);
    char *p = (char *)base;
    ScWork W;
    W.flag = (int32_t *)p;
    W.bnd = (double2 *)(p + z.flag);
    W.act = (double2 *)(p + z.flag + z.bnd);
    W.part = (Acc *)(p + z.flag + z.bnd + z.act);
    return W;
}

// The instance's own ScWork (allocated on first use, kept).
static int sc_work_own(bp_instance *h, ScWork &W) {
    if (int rc = h->sc_work.grow(sc_work_size(h).total(), h->bytes)) return rc;
    W = sc_work_at(h, h->sc_work.p);
    return 0;
}

// Chunk table of the rows longer than 1024 nonzeros (the block and heavy
// bins) from the cold-start row order `cold` (host): rows, their first
// chunk and the (row, chunk, chunks) records.  Built with the row bins.
static int sc_tables(bp_instance *h, const std::vector<int32_t> &cold, hipStream_t st) {
    std::vector<int32_t> rows;
    std::vector<int64_t> first(1, 0);
    std::vector<int4> chunks;
    for (int64_t t = h->bin_start[BIN_BLOCK]; t < h->bin_start[NBIN]; ++t) {
        const int32_t k = cold[t];
        const int32_t nch = (int32_t)((h->row_len[k] + SC_CHUNK - 1) / SC_CHUNK);
        for (int32_t c = 0; c < nch; ++c) chunks.push_back(make_int4(k, c, nch, 0));
        rows.push_back(k);
        first.push_back((int64_t)chunks.size());
    }
    h->sc_nlong = (int64_t)rows.size();
    h->sc_nchunks = (int64_t)chunks.size();
    int rc;
    if ((rc = h->sc_rows.alloc(std::max<size_t>(rows.size(), 1) * 4, h->bytes))) return rc;
    if ((rc = h->sc_first.alloc(first.size() * 8, h->bytes))) return rc;
    if ((rc = h->sc_chunks.alloc(std::max<size_t>(chunks.size(), 1) * sizeof(int4), h->bytes))) return rc;
    if (!rows.empty()) {
        HIPTRY(hipMemcpyAsync(h->sc_rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(h->sc_chunks.p, chunks.data(), chunks.size() * sizeof(int4),
                              hipMemcpyHostToDevice, st));
    }
    HIPTRY(hipMemcpyAsync(h->sc_first.p, first.data(), first.size() * 8, hipMemcpyHostToDevice, st));
    return 0;
}

// The exact activity of every row at the packed bounds W.bnd: the slacks
// into W.act and, when full is not null, the whole activities into full.
static int sc_rows_run(bp_instance *h, const ScWork &W, RowSums *full, hipStream_t st);

// Bounds in (NaN rejected), then the exact activity of every row, into W.
static int sc_rows_pass(bp_instance *h, const double *lb, const double *ub, const ScWork &W,
                        hipStream_t st) {
    const int64_t n = h->n;
    if (n > 0) {
        k_pack<<<grid_for(n), 256, 0, st>>>(lb, ub, W.bnd, n, 1);
        k_fill_i32<<<1, 64, 0, st>>>(W.flag, 0, 1);
        k_sc_nan<<<grid_for(n), 256, 0, st>>>(W.bnd, n, W.flag);
        HIPTRY(hipGetLastError());
        int32_t bad = 0;
        HIPTRY(hipMemcpyAsync(&bad, W.flag, 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (bad) return fail(BP_EINVAL, "NaN bound");
    }
    return sc_rows_run(h, W, nullptr, st);
}

static int sc_rows_run(bp_instance *h, const ScWork &W, RowSums *full, hipStream_t st) {
    const DInst I = dinst_of(h);
    const int32_t *cold = h->cold_rows.as<int32_t>();
    ScRowsWork R;
    R.chunks = h->sc_chunks.as<int4>();
    R.nchunks = h->sc_nchunks;
    R.start[0] = 0;
    R.start[1] = h->sc_nchunks;
    for (int j = 0; j < NLIGHT; ++j) {
        const int b = NLIGHT - 1 - j;
        const int64_t G = b >= 6 ? 64 : (int64_t)1 << b;
        R.rows[b] = cold + h->bin_start[b];
        R.count[b] = h->bin_count[b];
        R.start[2 + j] = R.start[1 + j] + (R.count[b] * G + WG - 1) / WG;
    }
    const int64_t units = R.start[NLIGHT + 1];
    if (units > 0)
        k_sc_rows<<<(int)std::min<int64_t>(units, 8192), WG, 0, st>>>(I, W.bnd, R, W.part, W.act,
                                                                      full);
    if (h->sc_nlong > 0)
        k_sc_combine<<<(int)std::min<int64_t>((h->sc_nlong + 3) / 4, 4096), WG, 0, st>>>(
            I, W.bnd, h->sc_rows.as<int32_t>(), h->sc_first.as<int64_t>(), h->sc_nlong, W.part,
            W.act, full);
    HIPTRY(hipGetLastError());
    return 0;
}

// Bitonic sort of kpad (a power of two) keys: sizes up to one tile entirely
// in LDS; each larger size runs the steps whose partners are a tile or more
// apart in global memory, then the rest in LDS.
static void sc_sort(ScKey *keys, int64_t kpad, hipStream_t st) {
    const int64_t tile = std::min<int64_t>(kpad, SC_TILE);
    const int tiles = (int)std::min<int64_t>(kpad / tile, 4096);
    if (kpad > 1) k_sc_bitonic_tile<<<tiles, SC_TILE_THREADS, 0, st>>>(keys, kpad, 2, tile, 1);
    for (int64_t size = 2 * tile; size <= kpad; size <<= 1) {
        for (int64_t stride = size >> 1; stride >= tile; stride >>= 1)
            k_sc_bitonic<<<grid_for(kpad), 256, 0, st>>>(keys, kpad, size, stride);
        k_sc_bitonic_tile<<<tiles, SC_TILE_THREADS, 0, st>>>(keys, kpad, size, size, tile >> 1);
    }
}

// Scores at lb/ub with the work buffers W (shared by bp_scores and
// bp_scores_noalloc).
static int sc_scores(bp_instance *h, const double *lb, const double *ub, bp_scores_out *out,
                     const ScWork &W, hipStream_t st) {
    if (int rc = sc_rows_pass(h, lb, ub, W, st)) return rc;
    if (h->n > 0)
        k_sc_vars<<<grid_for(h->n), 256, 0, st>>>(dinst_of(h), W.bnd, h->col_val.as<double>(), W.act,
                                                   h->opt.feastol, out->nviol, out->maxviol,
                                                   out->minunit, out->slack_score);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    return BP_OK;
}

extern "C" int bp_scores(bp_instance *h, const double *lb, const double *ub, bp_scores_out *out,
                         void *stream) {
    BP_RANGE("bp_scores");
    BP_TABLES_CHECK(h);
    if (!h || !out) return fail(BP_EINVAL, "null argument");
    if (h->n > 0 && (!lb || !ub)) return fail(BP_EINVAL, "null bounds");
    hipStream_t st = as_stream(stream);
    ScWork W;
    if (int rc = sc_work_own(h, W)) return rc;
    return sc_scores(h, lb, ub, out, W, st);
}

// ---------------------------------------------------------------------------
// Scores without device allocation.  The work buffers live in one static
// device array; each device that runs the library holds its own copy for
// the life of the process.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns, taken once per device
// on the first call there.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[BP_SCORES_NOALLOC_MAX_BYTES];

static const int SCRATCH_MAX_DEVICES = 64;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (taken on first use).
static int scratch_ptr(void **out) {
    int dev = -1;
    HIPTRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(BP_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

extern "C" int bp_scores_noalloc(bp_instance *h, const double *lb, const double *ub,
                                 bp_scores_out *out, void *stream) {
    if (!h || !out) return fail(BP_EINVAL, "null argument");
    BP_TABLES_CHECK(h);
    if (h->n > 0 && (!lb || !ub)) return fail(BP_EINVAL, "null bounds");
    const size_t need = sc_work_size(h).total();
    if (need > (size_t)BP_SCORES_NOALLOC_MAX_BYTES)
        return fail(BP_EINVAL, "bp_scores_noalloc: the instance needs " + std::to_string(need) +
                                   " bytes of work space, more than the " +
                                   std::to_string((long long)BP_SCORES_NOALLOC_MAX_BYTES) +
                                   " the static array holds");
    void *base = nullptr;
    if (int rc = scratch_ptr(&base)) return rc;
    return sc_scores(h, lb, ub, out, sc_work_at(h, base), as_stream(stream));
}

extern "C" int bp_probe_order(bp_instance *h, const double *lb, const double *ub,
                              const int32_t *vars, int32_t k, int32_t *order, void *stream) {
    BP_RANGE("bp_probe_order");
    BP_TABLES_CHECK(h);
    if (!h || k < 0) return fail(BP_EINVAL, "bad argument");
    if (k > 0 && (!vars || !order)) return fail(BP_EINVAL, "null argument");
    if (h->n > 0 && (!lb || !ub)) return fail(BP_EINVAL, "null bounds");
    hipStream_t st = as_stream(stream);
    if (k > 0)
        if (int rc = check_ids(h, vars, k, st)) return rc;
    ScWork W;
    if (int rc = sc_work_own(h, W)) return rc;
    if (int rc = sc_rows_pass(h, lb, ub, W, st)) return rc;
    if (k == 0) return BP_OK;
    const int64_t n = h->n;
    // nviol | maxviol | minunit of every variable
    if (int rc = h->sc_tmp.grow((size_t)n * 20, h->bytes)) return rc;
    double *mv = h->sc_tmp.as<double>();
    double *mu = mv + n;
    int32_t *nv = (int32_t *)(mu + n);
    k_sc_vars<<<grid_for(n), 256, 0, st>>>(dinst_of(h), W.bnd, h->col_val.as<double>(), W.act,
                                           h->opt.feastol, nv, mv, mu, nullptr);
    int64_t kpad = 1;
    while (kpad < k) kpad <<= 1;
    if (int rc = h->sc_keys.grow((size_t)kpad * sizeof(ScKey), h->bytes)) return rc;
    ScKey *keys = h->sc_keys.as<ScKey>();
    k_sc_keys<<<grid_for(kpad), 256, 0, st>>>(vars, k, kpad, nv, mv, mu, keys);
    sc_sort(keys, kpad, st);
    k_sc_order_out<<<grid_for(k), 256, 0, st>>>(keys, k, order);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    return BP_OK;
}
