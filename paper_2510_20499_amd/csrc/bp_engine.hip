// bp_engine.hip -- host runtime and C ABI of libbp.so (see include/bp.h).
//
// bp_load validates and uploads an instance and bins its rows by length.
// An Engine holds the per-slot work buffers for up to `cap_slots` bound
// vectors of one instance; propagate, propagate_batch and probe all run the
// same round kernels over it (bp_kernels.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/bp.h"
#include "bp_kernels.h"

using namespace bp;

// ------------------------------------------------------------------------
// Tracing: one roctx range per compute entry point call, named after it
// (rocprofv3 --marker-trace shows them around the call's kernels).
// ------------------------------------------------------------------------
struct RoctxRange {
    explicit RoctxRange(const char *name) { roctxRangePushA(name); }
    ~RoctxRange() { roctxRangePop(); }
    RoctxRange(const RoctxRange &) = delete;
    RoctxRange &operator=(const RoctxRange &) = delete;
};
#define BP_RANGE(name) RoctxRange bp_range_(name)

// ------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPTRY(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

// ------------------------------------------------------------------------
// Device buffers
// ------------------------------------------------------------------------
// Failure injection (bp_debug_fail_alloc): the number of device
// allocations still to succeed before one fails; 0 when disarmed.
static std::atomic<int64_t> g_fail_alloc{0};

static bool alloc_injected_failure() {
    int64_t k = g_fail_alloc.load();
    while (k > 0)
        if (g_fail_alloc.compare_exchange_weak(k, k - 1)) return k == 1;
    return false;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t n, int64_t &total) {
        if (p) {
            (void)hipFree(p);
            total -= (int64_t)bytes;
        }
        p = nullptr;
        bytes = 0;
        if (n == 0) n = 16;
        if (alloc_injected_failure())
            return fail(BP_ENOMEM, "injected failure of device allocation (" + std::to_string(n) +
                                       " bytes; bp_debug_fail_alloc)");
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(e == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE,
                        "hipMalloc(" + std::to_string(n) + "): " + hipGetErrorString(e));
        }
        bytes = n;
        total += (int64_t)n;
        return 0;
    }
    // Keeps the allocation when it is already large enough.
    int grow(size_t n, int64_t &total) {
        if (p && bytes >= n) return 0;
        return alloc(n, total);
    }
    template <class T>
    T *as() const {
        return (T *)p;
    }
};

// Per-slot capacities of an engine: variables and rows per slot (the largest
// instance whose vectors it holds), tasks per bin and heavy chunks per slot.
struct Shape {
    int64_t sn = 0, sm = 0;
    int64_t bin_cap[NBIN] = {0};
    int64_t heavy_chunks = 0;
    int64_t heavy_rows = 0;
    bool covers(const Shape &o) const {
        if (sn < o.sn || sm < o.sm || heavy_chunks < o.heavy_chunks || heavy_rows < o.heavy_rows)
            return false;
        for (int b = 0; b < NBIN; ++b)
            if (bin_cap[b] < o.bin_cap[b]) return false;
        return true;
    }
};

struct Engine {
    int32_t cap_slots = 0;
    int32_t track_dirty = 0;
    int32_t nstripe = 1;  // changed-list stripes (NSTRIPE for one slot)
    // scan rounds (engines of one slot) and incremental heavy rows (the
    // first inc_cap slots: INC_SLOTS, or every slot of a probe engine)
    DevBuf cbits, hhit, allhrec, hacc, hinf, hwid, hact, hcrec[2];
    int32_t inc_cap = 0;
    // every slot's heavy-row corrections are zero (a probe call ran to the
    // end: each retired job cleared its own)
    bool inc_clear = false;
    // rounds the last probe call ran (0: none yet)
    int32_t job_rounds = 0;
    Shape shape;
    int64_t bytes = 0;
    DevBuf bnd, cand, vflag, rflag, info, chg, dirty, dlist, dcount, ctl, touched, useen, filt;
    DevBuf q[2][NBIN], hrec[2], hpart, hrng;
    // Captured graphs of K rounds, keyed by their kernel arguments (held by
    // value): calls that alternate between argument sets (a propagation
    // and a probe on one instance) each keep theirs; the least recently
    // used is replaced.
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        int rounds = 0;
        bool jobs = false;
        Params P;
        JobIO io;
        uint64_t used = 0;
    };
    static constexpr int GRAPHS = 4;
    GraphEntry graphs[GRAPHS];
    uint64_t graph_clock = 0;
    ~Engine() {
        for (GraphEntry &g : graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
    }
};

#include "bp_lv.h"

struct bp_instance {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    bp_options opt;
    int64_t heavy_threshold = 8192;
    int32_t heavy_chunk = 4096;
    // device copies
    DevBuf row_ptr, col, val, side, col_ptr, col_row, col_val, vtype, rbin, cold_rows, base;
    DevBuf hidx_d;  // [m] heavy index of each row (-1: not heavy), bin order
    int64_t bytes = 0;
    bool have_base = false;
    int64_t base_version = 0;
    // probe staging (reused across calls)
    DevBuf st_var, st_lb, st_ub, st_off, st_cnt, scratch_i32;
    DevBuf st_status, st_rounds, st_nnz, st_jobs;  // per-job results and descriptors
    int64_t st_cap = 0;
    DevBuf box_d, ptr_d, idflag_d;  // per-call box check, changed offsets, id check
    // the heavy rows at the base bounds (incremental heavy rows of probe
    // slots): limbs [H][2][HL], infinite counts [H][2], widths [H]
    DevBuf hb_limb, hb_inf, hb_wid;
    int64_t hb_version = -1;  // base_version they were computed for
    // row bins (host)
    int64_t bin_count[NBIN] = {0};
    int64_t bin_start[NBIN + 1] = {0};
    int64_t heavy_chunks = 0;        // chunks of all heavy rows
    std::vector<int32_t> cold_hbase; // cold-start chunk base of each heavy row (bin order)
    std::vector<int32_t> row_len;    // host copy of the row lengths (re-binning)
    DevBuf cold_hbase_d;
    std::unique_ptr<Engine> eng;
    std::unique_ptr<LvEngine> lv;  // one-vector-per-lane batch engine
    // priority scores: the chunk table of the long rows (built with the row
    // bins), the per-call work (packed bounds, row activities, long-row
    // partials; allocated on first use) and sort buffers
    DevBuf sc_chunks, sc_rows, sc_first, sc_work, sc_tmp, sc_keys;
    int64_t sc_nchunks = 0, sc_nlong = 0;
    // bound-propagation rounding work buffers (rd_start: the box the
    // rounding started from, the repair's original box)
    DevBuf rd_order, rd_order2, rd_flags, rd_small, rd_S, rd_keys, rd_val, rd_keep, rd_mpos;
    DevBuf rd_mbox, rd_vk, rd_vl, rd_vu, rd_chg, rd_cpos, rd_bcnt, rd_start;
    // repair work buffers: row activities, candidates of a row, control
    // record, fixed flags, the box propagated from the original bounds
    DevBuf rp_sums, rp_cand, rp_ctl, rp_fixed, rp_pl, rp_pu;
    int64_t max_row_len = 0;
    // false while the row tables are being (re)built, and after a failed
    // rebuild: the instance then takes no further calls
    bool tables_ok = false;
    // stats
    bp_stats stats;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
    ~bp_instance() {
        eng.reset();
        lv.reset();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (ev2) (void)hipEventDestroy(ev2);
        if (ev3) (void)hipEventDestroy(ev3);
    }
};

extern "C" void bp_options_default(bp_options *o) {
    o->feastol = 1e-6;
    o->inttol = 1e-6;
    o->tau = 1e-3;
    o->max_rounds = 1000;
    o->flags = 0;
    o->heavy_threshold = 8192;
    o->rounds_per_launch = 16;
    o->probe_slots = 512;
    o->heavy_chunk = 1024;
    o->repair_calls = 0;
    o->repair_attempts = 8;
    o->repair_shifts = 64;
    o->lv_grid = 0;
}

extern "C" const char *bp_last_error(void) { return g_err.c_str(); }

extern "C" int bp_debug_fail_alloc(int64_t k) {
    if (k < 0) return fail(BP_EINVAL, "bp_debug_fail_alloc: negative count");
    g_fail_alloc.store(k);
    return BP_OK;
}

// ------------------------------------------------------------------------
// Small kernels: packing, checks, seeding
// ------------------------------------------------------------------------
__global__ void k_pack(const double *lb, const double *ub, double2 *bnd, int64_t n, int64_t B) {
    int64_t N = n * B;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x)
        bnd[j] = make_double2(canon0(lb[j]), canon0(ub[j]));
}

__global__ void k_unpack(const double2 *bnd, double *lb, double *ub, int64_t N) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        double2 b = bnd[j];
        lb[j] = b.x;
        ub[j] = b.y;
    }
}

__global__ void k_copy_bnd(const double2 *src, double2 *dst, int64_t N) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

// Step before the first round: a crossed or NaN box.  out[2*s] = smallest
// crossed var of slot s (NONE if none); out[2*s+1] = 1 if a NaN was seen.
__global__ void k_box_check(const double2 *bnd, const uint8_t *vtype, int64_t n, int32_t B,
                            double feastol, int32_t *out) {
    int64_t N = n * (int64_t)B;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        int s = (int)(j / n);
        int i = (int)(j - (int64_t)s * n);
        double2 b = bnd[j];
        if (isnan(b.x) || isnan(b.y)) atomicOr(&out[2 * s + 1], 1);
        double slack = vtype[i] ? 0.0 : feastol;
        if (b.x > b.y + slack) atomicMin(&out[2 * s], i);
    }
}

// Slots whose box is crossed before any round drain without running.
__global__ void k_box_drain(SlotInfo *info, const int32_t *box, int32_t B) {
    for (int j = threadIdx.x; j < B; j += blockDim.x)
        if (box[2 * j] != NONE) info[j].state = SLOT_DRAINING;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

__global__ void k_fill_cand(longlong2 *c, int64_t n) {
    const double INF = __builtin_inf();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        c[j] = make_longlong2(dkey(-INF), dkey(INF));
}

// Cold start of slots [s0, s0 + ns): every row of the instance, in bin
// order, into the queues of parity 0.  Slot j's rows of bin b sit at
// (j - s0) * count_b within the bin queue.
struct SeedAll {
    const int32_t *rows;       // rows grouped by bin
    int64_t start[NBIN + 1];
    const int32_t *hbase;      // cold chunk base of each heavy row (within one slot)
    int64_t chunks_per_slot;
    int32_t s0, ns;
};

__global__ void k_seed_all(Params P, SeedAll S) {
    int64_t m = S.start[NBIN];
    int64_t N = m * S.ns;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        int sl = (int)(j / m);
        int64_t r = j - (int64_t)sl * m;
        int b = 0;
        while (r >= S.start[b + 1]) ++b;
        int64_t cnt = S.start[b + 1] - S.start[b];
        int64_t within = r - S.start[b];
        int64_t idx = (int64_t)sl * cnt + within;
        int s = S.s0 + sl;
        int row = S.rows[r];
        if (b == BIN_HEAVY) {
            int64_t len = P.I.row_ptr[row + 1] - P.I.row_ptr[row];
            int32_t nch = (int32_t)((len + P.heavy_chunk - 1) / P.heavy_chunk);
            int64_t cb = (int64_t)sl * S.chunks_per_slot + S.hbase[within];
            for (int32_t c = 0; c < nch; ++c) P.hrec[0][cb + c] = make_int4(s, row, c, nch);
        } else {
            P.q[0][b][idx] = ((uint64_t)(uint32_t)s << 32) | (uint32_t)row;
        }
    }
}

// Chunk records of every heavy row in the cold-start layout (slot 0): the
// fixed list a scan round walks.
__global__ void k_fill_allhrec(DInst I, const int32_t *hrows, const int32_t *hbase, int64_t nheavy,
                               int32_t chunk, int4 *out) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nheavy;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int32_t row = hrows[w];
        const int64_t len = I.row_ptr[row + 1] - I.row_ptr[row];
        const int32_t nch = (int32_t)((len + chunk - 1) / chunk);
        for (int32_t c = 0; c < nch; ++c) out[hbase[w] + c] = make_int4(0, row, c, nch);
    }
}

// Warm start: the rows of the listed variables of each slot.  Entry e of
// (slot, var) pairs; launched with whole waves.
__global__ void k_seed_vars(Params P, const int32_t *vars, const int64_t *ptr, int32_t s0,
                            int32_t ns, int64_t total, int heavy_threshold) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += stride) {
        int64_t e = base + threadIdx.x;
        bool has = e < total;
        int s = 0, i = 0;
        long long c0 = 0;
        uint32_t clen = 0;
        if (has) {
            // slot of entry e: ptr is non-decreasing over ns slots
            int lo = 0, hi = ns;
            while (hi - lo > 1) {
                int mid = (lo + hi) / 2;
                if (ptr[mid] <= e) lo = mid;
                else hi = mid;
            }
            s = s0 + lo;
            i = vars[e];
            c0 = P.I.col_ptr[i];
            clen = (uint32_t)(P.I.col_ptr[i + 1] - c0);
        }
        enqueue_columns<false>(P, 0, has, s, c0, clen);
    }
}

// After seeding: a slot's first round counts its queued rows (a cold start
// queues every row).
__global__ void k_seed_finish(Params P, int32_t s0, int32_t ns, int32_t max_rounds, int cold,
                              int32_t m, long long nnz) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        SlotInfo &S = P.info[s0 + j];
        if (S.state != SLOT_ACTIVE) continue;
        if (cold) {
            S.pending_rows = m;
            S.pending_nnz = nnz;
        }
        if (S.pending_rows == 0) {
            S.state = SLOT_FREE;
            S.status = 0;
        } else if (max_rounds <= 0) {
            S.state = SLOT_DRAINING;
            S.status = 2;
        } else {
            S.rounds = 1;
            S.nnz = S.pending_nnz;
            atomicAdd(&P.ctl->stat_rows, (unsigned long long)S.pending_rows);
            atomicAdd(&P.ctl->stat_nnz, S.pending_nnz);
            S.pending_rows = 0;
            S.pending_nnz = 0;
        }
    }
}

// ------------------------------------------------------------------------
// Host helpers
// ------------------------------------------------------------------------
static hipStream_t as_stream(void *s) { return (hipStream_t)s; }

static int grid_for(int64_t n, int per = 256) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

static int validate_options(const bp_options &o) {
    if (!(o.feastol >= 0.0) || !(o.inttol >= 0.0) || !(o.tau >= 0.0) || o.max_rounds < 0)
        return fail(BP_EINVAL, "bad options: tolerances must be >= 0 and max_rounds >= 0");
    return 0;
}

static int sc_tables(bp_instance *h, const std::vector<int32_t> &cold, hipStream_t st);

// Row bins (logarithmic radix binning, the paper's Section 2.1 load
// balancing) for the instance's heavy threshold and chunk size: the bin of
// every row, the cold-start row order grouped by bin, and the chunk table
// of the heavy rows.  Run at load and again when the autotuner changes the
// schedule.
static int bin_rows(bp_instance *h, hipStream_t st) {
    const int64_t m = h->m;
    h->tables_ok = false;
    h->hb_version = -1;  // the heavy rows change with the threshold
    for (int b = 0; b < NBIN; ++b) h->bin_count[b] = 0;
    std::vector<uint8_t> rbin(m);
    for (int64_t k = 0; k < m; ++k) {
        int b = row_bin(h->row_len[k], h->heavy_threshold);
        rbin[k] = (uint8_t)b;
        h->bin_count[b] += 1;
    }
    h->bin_start[0] = 0;
    for (int b = 0; b < NBIN; ++b) h->bin_start[b + 1] = h->bin_start[b] + h->bin_count[b];
    std::vector<int32_t> cold(m);
    {
        std::vector<int64_t> fill(h->bin_start, h->bin_start + NBIN);
        for (int64_t k = 0; k < m; ++k) cold[fill[rbin[k]]++] = (int32_t)k;
    }
    std::vector<int32_t> hidx(m, -1);
    for (int64_t j = h->bin_start[BIN_HEAVY]; j < h->bin_start[BIN_HEAVY + 1]; ++j)
        hidx[cold[j]] = (int32_t)(j - h->bin_start[BIN_HEAVY]);
    h->heavy_chunks = 0;
    h->cold_hbase.clear();
    for (int64_t j = h->bin_start[BIN_HEAVY]; j < h->bin_start[BIN_HEAVY + 1]; ++j) {
        int64_t len = h->row_len[cold[j]];
        h->cold_hbase.push_back((int32_t)h->heavy_chunks);
        h->heavy_chunks += (len + h->heavy_chunk - 1) / h->heavy_chunk;
    }
    int rc;
    HIPTRY(hipStreamSynchronize(st));  // the previous tables may still be in use
    if ((rc = h->rbin.alloc((size_t)m, h->bytes))) return rc;
    if ((rc = h->cold_rows.alloc((size_t)m * 4, h->bytes))) return rc;
    if ((rc = h->cold_hbase_d.alloc(h->cold_hbase.size() * 4, h->bytes))) return rc;
    if ((rc = h->hidx_d.alloc((size_t)m * 4, h->bytes))) return rc;
    if (m) {
        HIPTRY(hipMemcpyAsync(h->hidx_d.p, hidx.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(h->rbin.p, rbin.data(), (size_t)m, hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(h->cold_rows.p, cold.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
    }
    if (!h->cold_hbase.empty())
        HIPTRY(hipMemcpyAsync(h->cold_hbase_d.p, h->cold_hbase.data(), h->cold_hbase.size() * 4,
                              hipMemcpyHostToDevice, st));
    if ((rc = sc_tables(h, cold, st))) return rc;
    HIPTRY(hipStreamSynchronize(st));
    h->tables_ok = true;
    return 0;
}

// Entry points on an instance whose row tables were lost (an allocation
// failed while the autotuner re-binned its rows) fail with BP_ESTATE.  A
// null instance is left to the entry point's own argument check.
static int tables_check(const bp_instance *h) {
    if (!h || h->tables_ok) return 0;
    return fail(BP_ESTATE, "the instance's row tables were lost in a failed allocation; load it again");
}
#define BP_TABLES_CHECK(h)                       \
    do {                                         \
        if (int rc_ = tables_check(h)) return rc_; \
    } while (0)

extern "C" int bp_load(const bp_sparse *csr, const bp_sparse *csc, const double *row_lo,
                       const double *row_hi, const uint8_t *vartype, const bp_options *opt,
                       void *stream, bp_instance **out) {
    BP_RANGE("bp_load");
    g_err.clear();
    if (!csr || !row_lo || !row_hi || !vartype || !out)
        return fail(BP_EINVAL, "bp_load: null argument");
    *out = nullptr;
    const int64_t m = csr->m, n = csr->n, nnz = csr->nnz;
    if (m < 0 || n < 0 || nnz < 0 || m >= INT32_MAX || n >= INT32_MAX)
        return fail(BP_EINVAL, "bp_load: bad sizes");
    if (!csr->ptr || (nnz > 0 && (!csr->idx || !csr->val)))
        return fail(BP_EINVAL, "bp_load: null CSR arrays");
    bp_options o;
    if (opt) o = *opt;
    else bp_options_default(&o);
    if (int rc = validate_options(o)) return rc;
    if (o.heavy_threshold <= 0) o.heavy_threshold = 8192;
    if (o.heavy_threshold < 1024) o.heavy_threshold = 1024;
    if (o.rounds_per_launch <= 0) o.rounds_per_launch = 16;
    if (o.probe_slots <= 0) o.probe_slots = 512;
    if (o.heavy_chunk <= 0) o.heavy_chunk = 1024;
    if (o.repair_calls < 0) o.repair_calls = 0;
    if (o.repair_attempts <= 0) o.repair_attempts = 8;
    if (o.repair_shifts <= 0) o.repair_shifts = 64;
    if (o.lv_grid < 0) o.lv_grid = 0;
    o.heavy_chunk = (o.heavy_chunk + WG - 1) / WG * WG;
    // CSR validation
    if (csr->ptr[0] != 0 || csr->ptr[m] != nnz) return fail(BP_EINVAL, "CSR ptr must run from 0 to nnz");
    for (int64_t k = 0; k < m; ++k) {
        if (csr->ptr[k + 1] < csr->ptr[k]) return fail(BP_EINVAL, "CSR ptr decreases at row " + std::to_string(k));
        double lo = row_lo[k], hi = row_hi[k];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY)
            return fail(BP_EINVAL, "bad sides at row " + std::to_string(k));
        for (int64_t p = csr->ptr[k]; p < csr->ptr[k + 1]; ++p) {
            int32_t c = csr->idx[p];
            if (c < 0 || c >= n) return fail(BP_EINVAL, "column out of range in row " + std::to_string(k));
            if (p > csr->ptr[k] && c <= csr->idx[p - 1])
                return fail(BP_EINVAL, "columns not ascending/distinct in row " + std::to_string(k));
            double v = csr->val[p];
            if (!(v != 0.0) || std::isinf(v))
                return fail(BP_EINVAL, "zero, NaN or infinite coefficient in row " + std::to_string(k));
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (vartype[i] > 1) return fail(BP_EINVAL, "vartype must be 0 or 1");
    // CSC: build, or check a given one against the transpose.
    std::vector<int64_t> cptr(n + 1, 0);
    std::vector<int32_t> crow(nnz);
    std::vector<double> cval(nnz);
    for (int64_t p = 0; p < nnz; ++p) cptr[csr->idx[p] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) cptr[i + 1] += cptr[i];
    {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t k = 0; k < m; ++k)
            for (int64_t p = csr->ptr[k]; p < csr->ptr[k + 1]; ++p) {
                const int64_t e = fill[csr->idx[p]]++;
                crow[e] = (int32_t)k;
                cval[e] = csr->val[p];
            }
    }
    if (csc) {
        if (csc->m != m || csc->n != n || csc->nnz != nnz || !csc->ptr || (nnz && !csc->idx))
            return fail(BP_EINVAL, "CSC shape differs from CSR");
        for (int64_t i = 0; i <= n; ++i)
            if (csc->ptr[i] != cptr[i]) return fail(BP_EINVAL, "CSC is not the transpose of CSR");
        for (int64_t p = 0; p < nnz; ++p)
            if (csc->idx[p] != crow[p]) return fail(BP_EINVAL, "CSC is not the transpose of CSR");
        if (csc->val) {
            std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
            for (int64_t k = 0; k < m; ++k)
                for (int64_t p = csr->ptr[k]; p < csr->ptr[k + 1]; ++p)
                    if (csc->val[fill[csr->idx[p]]++] != csr->val[p])
                        return fail(BP_EINVAL, "CSC values differ from CSR");
        }
    }
    std::unique_ptr<bp_instance> h(new bp_instance());
    h->m = (int32_t)m;
    h->n = (int32_t)n;
    h->nnz = nnz;
    h->opt = o;
    h->heavy_threshold = o.heavy_threshold;
    h->heavy_chunk = o.heavy_chunk;
    memset(&h->stats, 0, sizeof(h->stats));
    h->row_len.resize(m);
    for (int64_t k = 0; k < m; ++k) {
        h->row_len[k] = (int32_t)(csr->ptr[k + 1] - csr->ptr[k]);
        h->max_row_len = std::max<int64_t>(h->max_row_len, h->row_len[k]);
    }
    std::vector<double> side(2 * m);
    for (int64_t k = 0; k < m; ++k) {
        side[2 * k] = row_lo[k] == 0.0 ? 0.0 : row_lo[k];
        side[2 * k + 1] = row_hi[k] == 0.0 ? 0.0 : row_hi[k];
    }
    hipStream_t st = as_stream(stream);
    int64_t &B = h->bytes;
    int rc;
#define ALLOC_UP(buf, hostptr, nbytes)                                                      \
    do {                                                                                    \
        if ((rc = h->buf.alloc((nbytes), B))) return rc;                                    \
        if ((nbytes) > 0) HIPTRY(hipMemcpyAsync(h->buf.p, (hostptr), (nbytes), hipMemcpyHostToDevice, st)); \
    } while (0)
    ALLOC_UP(row_ptr, csr->ptr, (size_t)(m + 1) * 8);
    ALLOC_UP(col, csr->idx, (size_t)nnz * 4);
    ALLOC_UP(val, csr->val, (size_t)nnz * 8);
    ALLOC_UP(side, side.data(), (size_t)m * 16);
    ALLOC_UP(col_ptr, cptr.data(), (size_t)(n + 1) * 8);
    ALLOC_UP(col_row, crow.data(), (size_t)nnz * 4);
    ALLOC_UP(col_val, cval.data(), (size_t)nnz * 8);
    ALLOC_UP(vtype, vartype, (size_t)n);
#undef ALLOC_UP
    if ((rc = bin_rows(h.get(), st))) return rc;
    if ((rc = h->base.alloc((size_t)n * 16, B))) return rc;
    HIPTRY(hipStreamSynchronize(st));
    HIPTRY(hipEventCreate(&h->ev0));
    HIPTRY(hipEventCreate(&h->ev1));
    HIPTRY(hipEventCreate(&h->ev2));
    HIPTRY(hipEventCreate(&h->ev3));
    *out = h.release();
    return BP_OK;
}

extern "C" void bp_free(bp_instance *h) { delete h; }

extern "C" int64_t bp_device_bytes(const bp_instance *h) {
    if (!h) return 0;
    return h->bytes + (h->eng ? h->eng->bytes : 0);
}

// ------------------------------------------------------------------------
// Engine allocation
// ------------------------------------------------------------------------
static Shape shape_of(const bp_instance *h) {
    Shape sh;
    sh.sn = h->n;
    sh.sm = h->m;
    for (int b = 0; b < NBIN; ++b) sh.bin_cap[b] = h->bin_count[b];
    sh.heavy_chunks = h->heavy_chunks;
    sh.heavy_rows = h->bin_count[BIN_HEAVY];
    return sh;
}

// (Re)allocate `E` for `slots` bound vectors of shape `sh`; dirty: with the
// overlay bookkeeping of jobs; count: with the distinct-record bitmap;
// inc_all: incremental heavy-row accumulators for every slot (probe slots),
// not only the first INC_SLOTS.
static int engine_alloc(std::unique_ptr<Engine> &eng, const Shape &sh, int32_t slots, bool dirty,
                        bool count, hipStream_t st, bool inc_all = false) {
    if (eng && eng->cap_slots >= slots && eng->shape.covers(sh) && (!dirty || eng->track_dirty) &&
        (!count || eng->touched.p) && (!inc_all || eng->inc_cap >= slots))
        return 0;
    eng.reset();
    std::unique_ptr<Engine> E(new Engine());
    E->cap_slots = slots;
    E->track_dirty = dirty ? 1 : 0;
    E->shape = sh;
    const int64_t n = std::max<int64_t>(sh.sn, 1), m = std::max<int64_t>(sh.sm, 1), S = slots;
    const int64_t nw_var = (n + 31) / 32, nw_row = (m + 31) / 32;
    int64_t &B = E->bytes;
    int rc;
    if ((rc = E->bnd.alloc((size_t)S * n * 16, B))) return rc;
    if ((rc = E->cand.alloc((size_t)S * n * 16, B))) return rc;
    if ((rc = E->vflag.alloc((size_t)S * nw_var * 4, B))) return rc;
    if ((rc = E->rflag.alloc((size_t)S * nw_row * 4, B))) return rc;
    if ((rc = E->info.alloc((size_t)S * sizeof(SlotInfo), B))) return rc;
    E->nstripe = S == 1 ? NSTRIPE : 1;
    if ((rc = E->chg.alloc((size_t)E->nstripe * S * n * 8, B))) return rc;
    if (S == 1) {
        if ((rc = E->cbits.alloc((size_t)2 * nw_var * 4, B))) return rc;
        if ((rc = E->hhit.alloc((size_t)m * 4, B))) return rc;
    }
    if ((rc = E->allhrec.alloc((size_t)std::max<int64_t>(sh.heavy_chunks, 1) * sizeof(int4), B))) return rc;
    if (sh.heavy_rows > 0) {
        // incremental heavy rows of the first INC_SLOTS slots, or of all
        const int64_t IS = inc_all ? S : std::min<int64_t>(S, INC_SLOTS);
        const int64_t H = sh.heavy_rows * IS;
        const int64_t HC = std::max<int64_t>(sh.heavy_chunks, 1) * IS;
        E->inc_cap = (int32_t)IS;
        if ((rc = E->hacc.alloc((size_t)H * 2 * HL * 8, B)) || (rc = E->hinf.alloc((size_t)H * 8, B)) ||
            (rc = E->hwid.alloc((size_t)H * 8, B)) || (rc = E->hact.alloc((size_t)H * 16, B)) ||
            (rc = E->hcrec[0].alloc((size_t)HC * sizeof(int4), B)) ||
            (rc = E->hcrec[1].alloc((size_t)HC * sizeof(int4), B)))
            return rc;
    }
    if ((rc = E->ctl.alloc(sizeof(Ctl), B))) return rc;
    for (int par = 0; par < 2; ++par) {
        for (int b = 0; b < BIN_HEAVY; ++b)
            if ((rc = E->q[par][b].alloc((size_t)S * sh.bin_cap[b] * 8, B))) return rc;
        if ((rc = E->hrec[par].alloc((size_t)S * sh.heavy_chunks * sizeof(int4), B))) return rc;
    }
    if ((rc = E->hpart.alloc((size_t)S * sh.heavy_chunks * 2 * sizeof(Acc), B))) return rc;
    if ((rc = E->hrng.alloc((size_t)S * sh.heavy_chunks * sizeof(double), B))) return rc;
    if (count) {
        if ((rc = E->touched.alloc((size_t)S * nw_var * 4, B))) return rc;
        HIPTRY(hipMemsetAsync(E->touched.p, 0, E->touched.bytes, st));
        if ((rc = E->useen.alloc((size_t)nw_row * 4, B))) return rc;
        HIPTRY(hipMemsetAsync(E->useen.p, 0, E->useen.bytes, st));
    }
    if (dirty) {
        if ((rc = E->filt.alloc((size_t)S * FILT_WORDS * 4, B))) return rc;
        HIPTRY(hipMemsetAsync(E->filt.p, 0, E->filt.bytes, st));
        if ((rc = E->dirty.alloc((size_t)S * nw_var * 4, B))) return rc;
        if ((rc = E->dlist.alloc((size_t)S * n * 4, B))) return rc;
        if ((rc = E->dcount.alloc((size_t)S * 4, B))) return rc;
        HIPTRY(hipMemsetAsync(E->dirty.p, 0, E->dirty.bytes, st));
        HIPTRY(hipMemsetAsync(E->dcount.p, 0, E->dcount.bytes, st));
    }
    HIPTRY(hipMemsetAsync(E->vflag.p, 0, E->vflag.bytes, st));
    HIPTRY(hipMemsetAsync(E->rflag.p, 0, E->rflag.bytes, st));
    HIPTRY(hipMemsetAsync(E->info.p, 0, E->info.bytes, st));
    k_fill_cand<<<grid_for(S * n), 256, 0, st>>>(E->cand.as<longlong2>(), S * n);
    HIPTRY(hipGetLastError());
    eng = std::move(E);
    return 0;
}

static int engine_ensure(bp_instance *h, int32_t slots, bool dirty, hipStream_t st,
                         bool inc_all = false) {
    return engine_alloc(h->eng, shape_of(h), slots, dirty, (h->opt.flags & BP_FLAG_COUNT_VARS) != 0,
                        st, inc_all);
}

static DInst dinst_of(const bp_instance *h) {
    DInst I;
    I.m = h->m;
    I.n = h->n;
    I.row_ptr = h->row_ptr.as<int64_t>();
    I.col = h->col.as<int32_t>();
    I.val = h->val.as<double>();
    I.side = h->side.as<double2>();
    I.col_ptr = h->col_ptr.as<int64_t>();
    I.col_row = h->col_row.as<int32_t>();
    I.vtype = h->vtype.as<uint8_t>();
    I.rbin = h->rbin.as<uint8_t>();
    I.base = h->base.as<double2>();
    I.hidx = h->hidx_d.as<int32_t>();
    I.cval = h->col_val.as<double>();
    const bool hb = h->hb_version == h->base_version && h->hb_limb.p;
    I.hblimb = hb ? h->hb_limb.as<long long>() : nullptr;
    I.hbinf = hb ? h->hb_inf.as<int32_t>() : nullptr;
    I.hbwid = hb ? h->hb_wid.as<double>() : nullptr;
    return I;
}

// Kernel arguments for an engine; the instance fields are set by the caller.
static Params engine_params(const Engine &E, const bp_options &opt, int32_t heavy_chunk,
                            int32_t nslots) {
    Params P;
    memset(&P, 0, sizeof(P));
    P.feastol = opt.feastol;
    P.inttol = opt.inttol;
    P.tau = opt.tau;
    P.heavy_chunk = heavy_chunk;
    P.force_exact = (opt.flags & BP_FLAG_FORCE_EXACT) ? 1 : 0;
    P.nslots = nslots;
    P.sn = (int32_t)std::max<int64_t>(E.shape.sn, 1);
    P.snw = (int32_t)((P.sn + 31) / 32);
    P.srw = (int32_t)((std::max<int64_t>(E.shape.sm, 1) + 31) / 32);
    P.bnd = E.bnd.as<double2>();
    P.cand = E.cand.as<longlong2>();
    P.vflag = E.vflag.as<uint32_t>();
    P.rflag = E.rflag.as<uint32_t>();
    P.info = E.info.as<SlotInfo>();
    for (int par = 0; par < 2; ++par) {
        for (int b = 0; b < NBIN; ++b) P.q[par][b] = E.q[par][b].as<uint64_t>();
        P.hrec[par] = E.hrec[par].as<int4>();
    }
    P.hpart = E.hpart.as<Acc>();
    P.hrng = E.hrng.as<double>();
    P.chg = E.chg.as<uint64_t>();
    P.nstripe = E.nstripe;
    P.chg_stride = (int64_t)E.cap_slots * P.sn;
    P.ctl = E.ctl.as<Ctl>();
    P.touched = (opt.flags & BP_FLAG_COUNT_VARS) ? E.touched.as<uint32_t>() : nullptr;
    P.useen = (opt.flags & BP_FLAG_COUNT_VARS) ? E.useen.as<uint32_t>() : nullptr;
    P.overlay = 0;  // jobs read bounds as an overlay on the base
    P.filt = E.filt.as<uint32_t>();
    P.dirty = E.dirty.as<uint32_t>();
    P.dlist = E.dlist.as<int32_t>();
    P.dcount = E.dcount.as<int32_t>();
    return P;
}

static Params make_params(const bp_instance *h, int32_t nslots) {
    Params P = engine_params(*h->eng, h->opt, h->heavy_chunk, nslots);
    P.I = dinst_of(h);
    P.multi = 0;
    P.insts = nullptr;
    return P;
}

// A round with at least n / BP_INC_DIV changed variables hands the heavy-row
// accumulators to a rebuild in the next round instead of correcting them.
#ifndef BP_INC_DIV
#define BP_INC_DIV 256
#endif
static const int GRID_ROWS = 2048;
static const int GRID_HEAVY = 1024;
static const int GRID_APPLY = 512;

static int launch_round(bp_instance *h, const Params &P, const JobIO *io, hipStream_t st,
                        bool timed) {
    if (timed) {
        // Start/stop events recorded by the dispatch of k_rows itself, so the
        // interval is the kernel's execution (no dispatch latency).
        hipExtLaunchKernelGGL(k_rows<false>, dim3(GRID_ROWS), dim3(WG), 0, st, h->ev0, h->ev1, 0, P);
    } else {
        k_rows<false><<<GRID_ROWS, WG, 0, st>>>(P);
    }
    if (!P.inc_base) k_heavy<false><<<GRID_HEAVY, WG, 0, st>>>(P);  // job slots: decided by the heads
    if (timed) hipExtLaunchKernelGGL(k_apply<false>, dim3(GRID_APPLY), dim3(WG), 0, st, h->ev2, h->ev3, 0, P);
    else k_apply<false><<<GRID_APPLY, WG, 0, st>>>(P);
    if (io) k_end<END_WG><<<1, END_WG, 0, st>>>(P);
    else k_end<WG><<<1, WG, 0, st>>>(P);
    if (io) k_retire<false><<<std::min(P.nslots, 4096), WG, 0, st>>>(P, *io);
    HIPTRY(hipGetLastError());
    return 0;
}

// Run rounds until every slot is finished (and, when probing, every job).
static int run_rounds(bp_instance *h, const Params &P, const JobIO *io, int64_t limit,
                      hipStream_t st) {
    Engine &E = *h->eng;
    Ctl hc;
    const bool timed = (h->opt.flags & BP_FLAG_TIME_KERNELS) != 0;
    const bool host_rounds = timed || (h->opt.flags & BP_FLAG_HOST_ROUNDS) != 0;
    // Rounds per graph: rounds_per_launch, or for probe calls the smallest
    // power of two from 8 up that covered the last call's rounds, if less
    // (rounds after the last one still cost their launches).
    int K = std::max(1, (int)h->opt.rounds_per_launch);
    if (io && E.job_rounds > 0) {
        int k = 8;
        while (k < E.job_rounds && k < K) k *= 2;
        K = std::min(K, k);
    }
    int64_t launched = 0;
    for (;;) {
        if (host_rounds) {
            if (int rc = launch_round(h, P, io, st, timed)) return rc;
            launched += 1;
            if (timed) {
                HIPTRY(hipEventSynchronize(h->ev1));
                float ms = 0.f;
                HIPTRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
                h->stats.ms += ms;
                h->stats.launches += 1;
                HIPTRY(hipEventSynchronize(h->ev3));
                HIPTRY(hipEventElapsedTime(&ms, h->ev2, h->ev3));
                h->stats.apply_ms += ms;
            }
        } else {
            Engine::GraphEntry *G = nullptr;
            for (Engine::GraphEntry &g : E.graphs)
                if (g.exec && g.rounds == K && g.jobs == (io != nullptr) &&
                    memcmp(&g.P, &P, sizeof(Params)) == 0 && (!io || memcmp(&g.io, io, sizeof(JobIO)) == 0))
                    G = &g;
            if (!G) {
                G = &E.graphs[0];
                for (Engine::GraphEntry &g : E.graphs)
                    if (!g.exec || g.used < G->used) G = &g;
                if (G->exec) {
                    (void)hipGraphExecDestroy(G->exec);
                    G->exec = nullptr;
                }
                hipStream_t cs;
                HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                for (int r = 0; r < K; ++r) {
                    k_rows<false><<<GRID_ROWS, WG, 0, cs>>>(P);
                    // job slots' heavy rows are decided by their heads
                    if (!P.inc_base) k_heavy<false><<<GRID_HEAVY, WG, 0, cs>>>(P);
                    k_apply<false><<<GRID_APPLY, WG, 0, cs>>>(P);
                    if (io) k_end<END_WG><<<1, END_WG, 0, cs>>>(P);
                    else k_end<WG><<<1, WG, 0, cs>>>(P);
                    if (io) k_retire<false><<<std::min(P.nslots, 4096), WG, 0, cs>>>(P, *io);
                }
                hipGraph_t g;
                HIPTRY(hipStreamEndCapture(cs, &g));
                hipError_t e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                (void)hipStreamDestroy(cs);
                if (e != hipSuccess) G->exec = nullptr;
                HIPTRY(e);
                G->rounds = K;
                G->jobs = io != nullptr;
                G->P = P;
                if (io) G->io = *io;
            }
            G->used = ++E.graph_clock;
            HIPTRY(hipGraphLaunch(G->exec, st));
            launched += K;
        }
        HIPTRY(hipMemcpyAsync(&hc, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (hc.done) break;
        if (launched > limit) return fail(BP_EDEVICE, "round loop did not terminate");
    }
    if (io) E.job_rounds = (int32_t)std::min<uint32_t>(hc.round, 1u << 30);
    h->stats.rows += (int64_t)hc.stat_rows;
    h->stats.nnz += (int64_t)hc.stat_nnz;
    h->stats.vars_read += (int64_t)hc.stat_vars;
    h->stats.vars_written += (int64_t)hc.stat_written;
    h->stats.rows_kept += (int64_t)hc.stat_kept_rows;
    h->stats.nnz_kept += (int64_t)hc.stat_kept_nnz;
    h->stats.apply_entries += (int64_t)hc.stat_apply_entries;
    h->stats.apply_colent += (int64_t)hc.stat_apply_colent;
    h->stats.apply_corr += (int64_t)hc.stat_apply_corr;
    h->stats.rows_union += (int64_t)hc.stat_urows;
    h->stats.nnz_union += (int64_t)hc.stat_unnz;
    return 0;
}


// Reset the slots [0, ns) to `state`.
__global__ void k_reset_slots(SlotInfo *info, int32_t ns, int32_t job0, int32_t state) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ns; j += gridDim.x * blockDim.x) {
        SlotInfo &S = info[j];
        S.state = state;
        S.retire = 0;
        S.status = 0;
        S.rounds = 0;
        S.row_bad_min = NONE;
        S.row_bad_count = 0;
        S.var_bad_min = NONE;
        S.pending_rows = 0;
        S.job = job0 + j;
        S.nnz = 0;
        S.pending_nnz = 0;
    }
}

static int start_slots(bp_instance *h, const Params &P, int32_t ns, hipStream_t st,
                       const int32_t *changed_idx, const int64_t *changed_ptr,
                       int64_t n_changed_total, bool cold) {
    Ctl c;
    memset(&c, 0, sizeof(c));
    c.max_rounds = (uint32_t)h->opt.max_rounds;
    c.nslots = (uint32_t)ns;
    c.hbuild[0] = P.inc ? 1u : 0u;  // the first round builds the heavy-row accumulators
    if (cold) {
        for (int b = 0; b < NBIN; ++b) c.qcount[0][b] = (uint32_t)(h->bin_count[b] * ns);
        c.hchunks[0] = (uint32_t)(h->heavy_chunks * ns);
    }
    HIPTRY(hipMemcpyAsync(P.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
    k_reset_slots<<<grid_for(ns), 256, 0, st>>>(P.info, ns, 0, SLOT_ACTIVE);
    if (cold) {
        SeedAll S;
        S.rows = h->cold_rows.as<int32_t>();
        for (int b = 0; b <= NBIN; ++b) S.start[b] = h->bin_start[b];
        S.hbase = h->cold_hbase_d.as<int32_t>();
        S.chunks_per_slot = h->heavy_chunks;
        S.s0 = 0;
        S.ns = ns;
        int64_t N = (int64_t)h->m * ns;
        if (N > 0) k_seed_all<<<grid_for(N), 256, 0, st>>>(P, S);
    } else if (n_changed_total > 0) {
        k_seed_vars<<<grid_for(n_changed_total), 256, 0, st>>>(
            P, changed_idx, changed_ptr, 0, ns, n_changed_total, (int)h->heavy_threshold);
    }
    k_seed_finish<<<grid_for(ns), 256, 0, st>>>(P, 0, ns, h->opt.max_rounds, cold ? 1 : 0, h->m,
                                                 (long long)h->nnz);
    HIPTRY(hipGetLastError());
    return 0;
}

// Mark the control block done if no slot is active (e.g. empty worklists).
__global__ void k_check_any_active(Params P, int32_t ns) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < ns; j += blockDim.x)
        if (P.info[j].state != SLOT_FREE) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        P.ctl->done = any ? 0u : 1u;
        P.ctl->active = any ? 1u : 0u;
    }
}

static void fill_result(const SlotInfo &S, int32_t box_bad, bp_result *r) {
    memset(r, 0, sizeof(*r));
    r->infeasible_row = -1;
    r->infeasible_var = -1;
    if (box_bad != NONE) {
        r->status = BP_INFEASIBLE;
        r->infeasible_var = box_bad;
        return;
    }
    r->status = S.status;
    r->rounds = S.rounds;
    r->nnz_propagated = S.nnz;
    if (S.status == BP_INFEASIBLE) {
        if (S.row_bad_count > 0) {
            r->n_infeasible_rows = S.row_bad_count;
            r->infeasible_row = S.row_bad_min;
        } else {
            r->infeasible_var = S.var_bad_min;
        }
    }
}

// Any id outside [0, n) sets *bad.
__global__ void k_check_ids(const int32_t *ids, int64_t count, int32_t n, int32_t *bad) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < count;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = ids[j];
        if (v < 0 || v >= n) atomicOr(bad, 1);
    }
}

// Changed-variable ids of a call checked on the device (BP_EINVAL if any
// is out of range); only a flag comes back to the host.
static int check_ids(bp_instance *h, const int32_t *ids, int64_t count, hipStream_t st) {
    if (int rc = h->idflag_d.grow(4, h->bytes)) return rc;
    int32_t zero = 0, bad = 0;
    HIPTRY(hipMemcpyAsync(h->idflag_d.p, &zero, 4, hipMemcpyHostToDevice, st));
    k_check_ids<<<grid_for(count), 256, 0, st>>>(ids, count, h->n, h->idflag_d.as<int32_t>());
    HIPTRY(hipGetLastError());
    HIPTRY(hipMemcpyAsync(&bad, h->idflag_d.p, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (bad) return fail(BP_EINVAL, "changed variable id out of range");
    return 0;
}

// Shared driver of bp_propagate (B = 1, base update) and bp_propagate_batch.
static int propagate_slots(bp_instance *h, int32_t Bv, double *lb, double *ub,
                           const int32_t *changed_idx, const int64_t *changed_ptr,
                           int64_t n_changed_total, bool cold, bp_result *res, hipStream_t st,
                           bool ids_known_valid = false) {
    const int64_t n = h->n;
    if (int rc = engine_ensure(h, Bv, false, st)) return rc;
    Params P = make_params(h, Bv);
    if (Bv == 1 && h->eng->cbits.p) {
        // one plain vector: large bound updates switch the next round to a
        // scan of every row
        Engine &E1 = *h->eng;
        P.scan_ok = 1;
        P.scan_min = (uint32_t)std::max<int64_t>(1, h->n / 8);
        P.cbits = E1.cbits.as<uint32_t>();
        P.hhit = E1.hhit.as<uint32_t>();
        P.allrows = h->cold_rows.as<int32_t>();
        for (int b = 0; b <= NBIN; ++b) P.allstart[b] = h->bin_start[b];
        HIPTRY(hipMemsetAsync(E1.cbits.p, 0, E1.cbits.bytes, st));
        HIPTRY(hipMemsetAsync(E1.hhit.p, 0, E1.hhit.bytes, st));
    }
    {
        // every heavy chunk (the list scan rounds and accumulator rebuilds
        // walk), and incremental heavy rows for one plain vector or a cold
        // start of up to INC_SLOTS
        Engine &E1 = *h->eng;
        const int64_t nheavy = h->bin_count[BIN_HEAVY];
        P.allhrec = E1.allhrec.as<int4>();
        P.allhchunks = (int32_t)h->heavy_chunks;
        // The first round builds every heavy row of every vector: worth it
        // for one vector, and for several on a cold start (where the first
        // round reads every row anyway); several warm vectors, as in the
        // rounding steps, recompute the few heavy rows they queue.
        if (nheavy > 0 && Bv <= INC_SLOTS && (Bv == 1 || cold) && E1.hacc.p &&
            !(h->opt.flags & BP_FLAG_FULL_ROWS)) {
            const size_t nh = (size_t)nheavy * Bv;
            P.inc = 1;
            P.nheavy = (int32_t)nheavy;
            P.inc_slots = Bv;
            P.hacc = E1.hacc.as<long long>();
            P.hinf = E1.hinf.as<int32_t>();
            P.hwid = E1.hwid.as<unsigned long long>();
            P.hact = E1.hact.as<double2>();
            P.hcrec[0] = E1.hcrec[0].as<int4>();
            P.hcrec[1] = E1.hcrec[1].as<int4>();
            P.inc_max = (uint32_t)std::max<int64_t>(64, (int64_t)h->n * Bv / BP_INC_DIV);
            // Limb bound: a build adds at most L pieces below 2^32 to a limb
            // of a row of L nonzeros, and a round at most 2L more (each of its
            // variables' old term out, new term in, once per side); after k
            // rounds |limb| < L 2^32 (1 + 2k), below 2^62 while 1 + 2k <
            // 2^30 / L.  Rebuilding at least that often keeps carry_round's
            // precondition whatever max_rounds is.
            {
                const int64_t L = std::max<int64_t>(h->max_row_len, 1);
                const int64_t k = ((int64_t(1) << 30) / L - 1) / 2;
                P.inc_period = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(k, 1 << 30));
            }
            HIPTRY(hipMemsetAsync(E1.hacc.p, 0, nh * 2 * HL * 8, st));
            HIPTRY(hipMemsetAsync(E1.hinf.p, 0, nh * 8, st));
            HIPTRY(hipMemsetAsync(E1.hwid.p, 0, nh * 8, st));
            E1.inc_clear = false;  // this call's accumulators are not cleared at its end
        }
        if (nheavy > 0 && (P.scan_ok || P.inc))
            k_fill_allhrec<<<grid_for(nheavy), 256, 0, st>>>(dinst_of(h), h->cold_rows.as<int32_t>() + h->bin_start[BIN_HEAVY],
                                                             h->cold_hbase_d.as<int32_t>(), nheavy, h->heavy_chunk,
                                                             E1.allhrec.as<int4>());
    }
    Engine &E = *h->eng;
    // Bounds in, box check.
    if (n > 0) k_pack<<<grid_for(n * Bv), 256, 0, st>>>(lb, ub, E.bnd.as<double2>(), n, Bv);
    DevBuf &boxd = h->box_d;
    if (int rc = boxd.grow((size_t)Bv * 8, h->bytes)) return rc;
    {
        // even entries: smallest crossed var; odd entries: NaN flags
        std::vector<int32_t> init(2 * (size_t)Bv);
        for (int32_t j = 0; j < Bv; ++j) {
            init[2 * j] = NONE;
            init[2 * j + 1] = 0;
        }
        HIPTRY(hipMemcpyAsync(boxd.p, init.data(), init.size() * 4, hipMemcpyHostToDevice, st));
    }
    if (n > 0)
        k_box_check<<<grid_for(n * Bv), 256, 0, st>>>(E.bnd.as<double2>(), h->vtype.as<uint8_t>(),
                                                      n, Bv, h->opt.feastol, boxd.as<int32_t>());
    HIPTRY(hipGetLastError());
    // Calls from inside the library (ids_known_valid: the bound-propagation
    // rounding) pass bounds its own kernels made, free of NaN: their crossed
    // boxes are handled on the device and read back with the results, which
    // spares a host round trip per call.
    std::vector<int32_t> box(2 * (size_t)Bv);
    if (!ids_known_valid) {
        HIPTRY(hipMemcpyAsync(box.data(), boxd.p, box.size() * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        for (int32_t j = 0; j < Bv; ++j)
            if (box[2 * j + 1]) return fail(BP_EINVAL, "NaN bound in vector " + std::to_string(j));
    }
    // Validate changed ids.
    if (!cold && n_changed_total > 0 && !ids_known_valid)
        if (int rc = check_ids(h, changed_idx, n_changed_total, st)) return rc;
    if (int rc = start_slots(h, P, Bv, st, changed_idx, changed_ptr, n_changed_total, cold)) return rc;
    // A slot whose box is already crossed is infeasible before any round;
    // its queued rows drain without running.
    if (ids_known_valid) {
        k_box_drain<<<1, 256, 0, st>>>(P.info, boxd.as<int32_t>(), Bv);
    } else {
        for (int32_t j = 0; j < Bv; ++j) {
            if (box[2 * j] == NONE) continue;
            int32_t dr = SLOT_DRAINING;
            HIPTRY(hipMemcpyAsync(&P.info[j].state, &dr, 4, hipMemcpyHostToDevice, st));
        }
    }
    k_check_any_active<<<1, 256, 0, st>>>(P, Bv);
    HIPTRY(hipGetLastError());
    if (int rc = run_rounds(h, P, nullptr, (int64_t)h->opt.max_rounds + 2, st)) return rc;
    std::vector<SlotInfo> info(Bv);
    HIPTRY(hipMemcpyAsync(info.data(), P.info, Bv * sizeof(SlotInfo), hipMemcpyDeviceToHost, st));
    if (ids_known_valid) HIPTRY(hipMemcpyAsync(box.data(), boxd.p, box.size() * 4, hipMemcpyDeviceToHost, st));
    if (n > 0) k_unpack<<<grid_for(n * Bv), 256, 0, st>>>(E.bnd.as<double2>(), lb, ub, n * Bv);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    for (int32_t j = 0; j < Bv; ++j) fill_result(info[j], box[2 * j], &res[j]);
    return 0;
}

extern "C" int bp_propagate(bp_instance *h, double *lb, double *ub, const int32_t *changed,
                            int64_t n_changed, bp_result *res, void *stream) {
    BP_RANGE("bp_propagate");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !res || (h->n > 0 && (!lb || !ub))) return fail(BP_EINVAL, "bp_propagate: null argument");
    hipStream_t st = as_stream(stream);
    bool cold = changed == nullptr;
    if (!cold && n_changed < 0) return fail(BP_EINVAL, "n_changed < 0");
    DevBuf &ptrd = h->ptr_d;
    if (!cold) {
        if (int rc = ptrd.grow(16, h->bytes)) return rc;
        int64_t p2[2] = {0, n_changed};
        HIPTRY(hipMemcpyAsync(ptrd.p, p2, 16, hipMemcpyHostToDevice, st));
    }
    int rc = propagate_slots(h, 1, lb, ub, changed, cold ? nullptr : ptrd.as<int64_t>(), cold ? 0 : n_changed, cold,
                             res, st);
    if (rc < 0) return rc;
    if (res->status == BP_OK && h->n > 0) {
        k_copy_bnd<<<grid_for(h->n), 256, 0, st>>>(h->eng->bnd.as<double2>(), h->base.as<double2>(), h->n);
        HIPTRY(hipGetLastError());
        HIPTRY(hipStreamSynchronize(st));
    }
    if (res->status == BP_OK) {
        h->have_base = true;
        h->base_version += 1;
    }
    return res->status;
}

#include "bp_lv_run.h"

extern "C" int bp_propagate_batch(bp_instance *h, int32_t B, double *lb, double *ub,
                                  const int64_t *changed_ptr, const int32_t *changed_idx,
                                  bp_result *res, void *stream) {
    BP_RANGE("bp_propagate_batch");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !res || B < 0 || (B > 0 && h->n > 0 && (!lb || !ub)))
        return fail(BP_EINVAL, "bp_propagate_batch: bad argument");
    if (B == 0) return BP_OK;
    hipStream_t st = as_stream(stream);
    bool cold = changed_ptr == nullptr;
    int64_t total = 0;
    std::vector<int64_t> ptr;
    if (!cold) {
        ptr.resize(B + 1);
        HIPTRY(hipMemcpyAsync(ptr.data(), changed_ptr, (B + 1) * 8, hipMemcpyDeviceToHost, as_stream(stream)));
        HIPTRY(hipStreamSynchronize(st));
        if (ptr[0] != 0) return fail(BP_EINVAL, "changed_ptr[0] must be 0");
        for (int32_t j = 0; j < B; ++j)
            if (ptr[j + 1] < ptr[j]) return fail(BP_EINVAL, "changed_ptr decreases");
        total = ptr[B];
        if (total > 0 && !changed_idx) return fail(BP_EINVAL, "changed_idx is null");
    }
    // Batches of LV_MIN_BATCH vectors or more run one vector per lane.
    if (B >= LV_MIN_BATCH && !(h->opt.flags & BP_FLAG_BATCH_SLOTS)) {
        int rc = lv_propagate(h, B, lb, ub, changed_idx, changed_ptr, ptr, cold, res, st);
        return rc < 0 ? rc : BP_OK;
    }
    int rc = propagate_slots(h, B, lb, ub, changed_idx, changed_ptr, total, cold, res, st);
    return rc < 0 ? rc : BP_OK;
}

extern "C" int bp_get_base(bp_instance *h, double *lb, double *ub, void *stream) {
    g_err.clear();
    if (!h || (h->n > 0 && (!lb || !ub))) return fail(BP_EINVAL, "bp_get_base: null argument");
    if (!h->have_base) return fail(BP_ESTATE, "no base: run a feasible bp_propagate first");
    hipStream_t st = as_stream(stream);
    if (h->n > 0) k_unpack<<<grid_for(h->n), 256, 0, st>>>(h->base.as<double2>(), lb, ub, h->n);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    return BP_OK;
}

extern "C" int bp_kernel_stats(bp_instance *h, bp_stats *out, int reset) {
    if (!h || !out) return fail(BP_EINVAL, "bp_kernel_stats: null argument");
    *out = h->stats;
    if (reset) memset(&h->stats, 0, sizeof(h->stats));
    return BP_OK;
}

// The heavy rows at the base bounds (one workgroup per row): each side's
// exact finite sum as carry-save limbs (every term's pieces added in LDS,
// the order-independent integer form of the incremental heavy rows), the
// counts of infinite contributions and the largest nonzero width.
__global__ void __launch_bounds__(WG) k_base_limbs(DInst I, const int32_t *hrows, int32_t H,
                                                   long long *limbs, int32_t *ninf_out, double *wid_out) {
    __shared__ long long L[2 * HL];
    __shared__ int32_t ninf[2];
    __shared__ unsigned long long wbits;
    for (int h = blockIdx.x; h < H; h += gridDim.x) {
        for (int j = threadIdx.x; j < 2 * HL; j += WG) L[j] = 0;
        if (threadIdx.x == 0) {
            ninf[0] = 0;
            ninf[1] = 0;
            wbits = 0ull;
        }
        __syncthreads();
        const int k = hrows[h];
        const int64_t p0 = I.row_ptr[k], p1 = I.row_ptr[k + 1];
        int nmin = 0, nmax = 0;
        double wmax = 0.0;
        const int iters = (int)((p1 - p0 + WG - 1) / WG);  // uniform: whole waves add together
        for (int it = 0; it < iters; ++it) {
            const int64_t p = p0 + threadIdx.x + (int64_t)it * WG;
            const bool in = p < p1;
            double tmin = 0.0, tmax = 0.0;
            if (in) {
                const double a = I.val[p];
                const double2 b = I.base[I.col[p]];
                const double bmin = a > 0.0 ? b.x : b.y;
                const double bmax = a > 0.0 ? b.y : b.x;
                if (isinf(bmin)) nmin += 1;
                else tmin = a * bmin;
                if (isinf(bmax)) nmax += 1;
                else tmax = a * bmax;
                wmax = fmax(wmax, nz_width(a, b.x, b.y));
            }
            inc_add_wave(L, tmin, in);
            inc_add_wave(L + HL, tmax, in);
        }
        if (nmin) atomicAdd(&ninf[0], nmin);
        if (nmax) atomicAdd(&ninf[1], nmax);
        if (wmax > 0.0) atomicMax(&wbits, (unsigned long long)__double_as_longlong(wmax));
        __syncthreads();
        for (int j = threadIdx.x; j < 2 * HL; j += WG) limbs[(size_t)h * 2 * HL + j] = L[j];
        if (threadIdx.x == 0) {
            ninf_out[2 * h] = ninf[0];
            ninf_out[2 * h + 1] = ninf[1];
            wid_out[h] = __longlong_as_double((long long)wbits);
        }
        __syncthreads();
    }
}

// The heavy rows of h at its base bounds (k_base_limbs), once per base.
static int base_limbs(bp_instance *h, hipStream_t st) {
    const int64_t H = h->bin_count[BIN_HEAVY];
    if (h->hb_version == h->base_version) return 0;
    if (H == 0) {
        h->hb_version = h->base_version;  // nothing to sum
        return 0;
    }
    if (int rc = h->hb_limb.grow((size_t)H * 2 * HL * 8, h->bytes)) return rc;
    if (int rc = h->hb_inf.grow((size_t)H * 8, h->bytes)) return rc;
    if (int rc = h->hb_wid.grow((size_t)H * 8, h->bytes)) return rc;
    k_base_limbs<<<(int)std::min<int64_t>(H, 4096), WG, 0, st>>>(
        dinst_of(h), h->cold_rows.as<int32_t>() + h->bin_start[BIN_HEAVY], (int32_t)H,
        h->hb_limb.as<long long>(), h->hb_inf.as<int32_t>(), h->hb_wid.as<double>());
    HIPTRY(hipGetLastError());
    h->hb_version = h->base_version;
    return 0;
}

// Incremental heavy rows over the base keep their limbs below carry_round's
// 2^62: the base limbs hold at most L pieces below 2^32 per limb (a row of L
// nonzeros), admission and each round of a job at most 2L more (old term
// out, new term in, once per variable and side), so after a job's
// r <= max_rounds rounds |limb| < L 2^32 (3 + 2r), in range while
// L (3 + 2 max_rounds) < 2^30.
static bool base_inc_ok(const bp_instance *h, int32_t max_rounds) {
    const int64_t L = std::max<int64_t>(h->max_row_len, 1);
    return L * (3 + 2 * (int64_t)max_rounds) < (int64_t(1) << 30);
}

// Probe variables must be integers with at least one finite base bound.
__global__ void k_check_probe_vars(const int32_t *vars, int32_t k, int32_t n, const uint8_t *vtype,
                                   const double2 *base, int32_t *bad) {
    const double INF = __builtin_inf();
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < k; t += gridDim.x * blockDim.x) {
        int j = vars[t];
        bool ok = j >= 0 && j < n;
        if (ok) {
            double2 b = base[j];
            ok = vtype[j] != 0 && (b.x > -INF || b.y < INF);
        }
        if (!ok) atomicMin(bad, t);
    }
}

// Done before the first round when no slot was admitted with work.
__global__ void k_probe_start_check(Params P) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < P.nslots; j += blockDim.x)
        if (P.info[j].state != SLOT_FREE) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0)
        P.ctl->done = (!any && P.ctl->next_job >= P.ctl->total_jobs) ? 1u : 0u;
}

static int ensure_buf(DevBuf &b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return 0;
    int64_t dummy = 0;
    return b.alloc(bytes, dummy);
}

extern "C" int bp_probe(bp_instance *h, const int32_t *vars, int32_t k, bp_probe_out *out,
                        void *stream) {
    BP_RANGE("bp_probe");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !out || k < 0 || (k > 0 && !vars)) return fail(BP_EINVAL, "bp_probe: bad argument");
    if (!out->off || out->cap < 0 || (k > 0 && (!out->status || !out->rounds || !out->nnz)))
        return fail(BP_EINVAL, "bp_probe: null output buffer");
    if (out->cap > 0 && (!out->var || !out->lb || !out->ub))
        return fail(BP_EINVAL, "bp_probe: null list buffer");
    if (!h->have_base) return fail(BP_ESTATE, "no base: run a feasible bp_propagate first");
    hipStream_t st = as_stream(stream);
    const int64_t n = h->n;
    const int64_t jobs = 2 * (int64_t)k;
    if (k == 0) {
        int64_t zero = 0;
        HIPTRY(hipMemcpyAsync(out->off, &zero, 8, hipMemcpyHostToDevice, st));
        HIPTRY(hipStreamSynchronize(st));
        out->required = 0;
        return BP_OK;
    }
    // Validate the variables on the device against the base.
    if (int rc = ensure_buf(h->scratch_i32, 16)) return rc;
    {
        int32_t none = NONE;
        HIPTRY(hipMemcpyAsync(h->scratch_i32.p, &none, 4, hipMemcpyHostToDevice, st));
        k_check_probe_vars<<<grid_for(k), 256, 0, st>>>(vars, k, h->n, h->vtype.as<uint8_t>(),
                                                        h->base.as<double2>(), h->scratch_i32.as<int32_t>());
        HIPTRY(hipGetLastError());
        int32_t bad = NONE;
        HIPTRY(hipMemcpyAsync(&bad, h->scratch_i32.p, 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (bad != NONE)
            return fail(BP_EINVAL, "probe variable at position " + std::to_string(bad) +
                                       " is not an integer with a finite base bound");
    }
    const int32_t S = (int32_t)std::min<int64_t>(std::max(1, h->opt.probe_slots), jobs);
    const int64_t H = h->bin_count[BIN_HEAVY];
    // Incremental heavy rows over the base while their limbs stay in range;
    // otherwise, or with FULL_ROWS, each slot's heavy rows are summed chunk
    // by chunk.
    const bool inc = H > 0 && !(h->opt.flags & BP_FLAG_FULL_ROWS) && base_inc_ok(h, h->opt.max_rounds);
    if (int rc = engine_ensure(h, S, true, st, inc)) return rc;
    Engine &E = *h->eng;
    if (inc)
        if (int rc = base_limbs(h, st)) return rc;
    // Probe slots read the base except where their dirty bits are set; a
    // retired probe clears its bits, so no slot needs initialising.
    // Staging for the implied lists.
    const int64_t cap = std::max<int64_t>(out->cap, 1);
    if (int rc = ensure_buf(h->st_var, (size_t)cap * 4)) return rc;
    if (int rc = ensure_buf(h->st_lb, (size_t)cap * 8)) return rc;
    if (int rc = ensure_buf(h->st_ub, (size_t)cap * 8)) return rc;
    if (int rc = ensure_buf(h->st_off, (size_t)jobs * 8)) return rc;
    if (int rc = ensure_buf(h->st_cnt, (size_t)jobs * 8)) return rc;
    // Library-owned copies keep the captured graph's arguments stable across calls.
    if (int rc = ensure_buf(h->st_status, (size_t)jobs)) return rc;
    if (int rc = ensure_buf(h->st_rounds, (size_t)jobs * 4)) return rc;
    if (int rc = ensure_buf(h->st_nnz, (size_t)jobs * 8)) return rc;
    if (int rc = ensure_buf(h->st_jobs, (size_t)jobs * sizeof(Job))) return rc;
    k_make_probe_jobs<<<grid_for(jobs), 256, 0, st>>>(vars, k, h->st_jobs.as<Job>());
    JobIO IO;
    memset(&IO, 0, sizeof(IO));
    IO.jobs = h->st_jobs.as<Job>();
    IO.status = h->st_status.as<int8_t>();
    IO.rounds = h->st_rounds.as<int32_t>();
    IO.nnz = h->st_nnz.as<int64_t>();
    IO.stage_off = h->st_off.as<int64_t>();
    IO.stage_cnt = h->st_cnt.as<int64_t>();
    IO.stage_var = h->st_var.as<int32_t>();
    IO.stage_lb = h->st_lb.as<double>();
    IO.stage_ub = h->st_ub.as<double>();
    IO.stage_cap = cap;
    Params P = make_params(h, S);
    P.overlay = 1;
    if (inc) {
        // every slot's corrections start at zero (a retired job clears its
        // own; this also drops what an interrupted call left)
        P.inc = 1;
        P.nheavy = (int32_t)H;
        P.inc_slots = S;
        P.hacc = E.hacc.as<long long>();
        P.hinf = E.hinf.as<int32_t>();
        P.hwid = E.hwid.as<unsigned long long>();
        P.hact = E.hact.as<double2>();
        P.hcrec[0] = E.hcrec[0].as<int4>();
        P.hcrec[1] = E.hcrec[1].as<int4>();
        P.inc_max = 0xffffffffu;  // never rebuilt
        P.inc_period = 0;
        P.inc_base = 1;
        if (!E.inc_clear) {
            HIPTRY(hipMemsetAsync(E.hacc.p, 0, (size_t)E.inc_cap * H * 2 * HL * 8, st));
            HIPTRY(hipMemsetAsync(E.hinf.p, 0, (size_t)E.inc_cap * H * 8, st));
        }
        E.inc_clear = false;  // until this call ends normally
    }
    Ctl c;
    memset(&c, 0, sizeof(c));
    c.max_rounds = (uint32_t)h->opt.max_rounds;
    c.nslots = (uint32_t)S;
    c.total_jobs = (uint32_t)jobs;
    HIPTRY(hipMemcpyAsync(P.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
    k_reset_slots<<<grid_for(S), 256, 0, st>>>(P.info, S, 0, SLOT_FREE);
    k_retire<false><<<std::min(S, 4096), WG, 0, st>>>(P, IO);  // first admissions
    k_probe_start_check<<<1, 256, 0, st>>>(P);
    HIPTRY(hipGetLastError());
    const int64_t limit = ((int64_t)h->opt.max_rounds + 2) * (jobs + 1);
    if (int rc = run_rounds(h, P, &IO, limit, st)) return rc;
    if (inc) E.inc_clear = true;  // every job retired
    Ctl hc;
    HIPTRY(hipMemcpyAsync(&hc, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    out->required = (int64_t)hc.stage_count;
    HIPTRY(hipMemcpyAsync(out->status, IO.status, (size_t)jobs, hipMemcpyDeviceToDevice, st));
    HIPTRY(hipMemcpyAsync(out->rounds, IO.rounds, (size_t)jobs * 4, hipMemcpyDeviceToDevice, st));
    HIPTRY(hipMemcpyAsync(out->nnz, IO.nnz, (size_t)jobs * 8, hipMemcpyDeviceToDevice, st));
    if (out->required > out->cap)
        return fail(BP_ECAPACITY, "implied lists need " + std::to_string(out->required) +
                                      " entries, capacity is " + std::to_string(out->cap));
    k_job_offsets<<<1, WG, 0, st>>>(IO.stage_cnt, out->off, jobs);
    k_job_gather<<<grid_for(jobs * 64, 256), 256, 0, st>>>(IO, out->off, jobs, out->var, out->lb,
                                                            out->ub);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    return BP_OK;
}

#include "bp_scores.h"
#include "bp_scores_run.h"
#include "bp_repair.h"
#include "bp_repair_run.h"
#include "bp_round.h"
#include "bp_round_run.h"
#include "bp_server.h"
#include "bp_tune.h"
