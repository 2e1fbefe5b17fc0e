// bp_server.h -- continuous-batching server (part of bp_engine.hip's
// translation unit; see include/bp.h for the C ABI).
//
// Requests become jobs: a probe request of k binaries is 2k probe jobs, a
// propagate request is one fixing job.  The served instances are grouped
// into classes by size, and each class has its own pool: an engine whose
// slots are sized for the class's largest instance, a device job list, a
// completion ring and a stream.  Each round's kernels of a pool process the
// tasks of its busy slots, and k_retire writes finished jobs' results,
// restores their slots and admits the next jobs.  The host appends newly
// submitted requests to their pool's list between graph launches, runs the
// pools' graphs side by side on their streams, and collects finished jobs
// from the rings.
#pragma once
#include <chrono>
#include <deque>
#include <numeric>
#include <unordered_map>

struct JobOut {
    int32_t job;
    int32_t status, rounds, n_bad_rows, bad_row, bad_var;
    int64_t nnz, stage_off, stage_cnt;
};

// Results of the finished jobs ring[r0 .. r1) into a compact array.
__global__ void k_collect(const JobIO IO, const uint32_t *ring, uint32_t r0, uint32_t r1, JobOut *out) {
    for (uint32_t t = r0 + blockIdx.x * blockDim.x + threadIdx.x; t < r1; t += gridDim.x * blockDim.x) {
        uint32_t p = ring[t];
        JobOut o;
        o.job = (int32_t)p;
        o.status = IO.status[p];
        o.rounds = IO.rounds[p];
        o.n_bad_rows = IO.n_bad_rows[p];
        o.bad_row = IO.bad_row[p];
        o.bad_var = IO.bad_var[p];
        o.nnz = IO.nnz[p];
        o.stage_off = IO.stage_off[p];
        o.stage_cnt = IO.stage_cnt[p];
        out[t - r0] = o;
    }
}

// Done before the next round when no slot is busy and no job waits.
__global__ void k_jobs_done_check(Params P) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < P.nslots; j += blockDim.x)
        if (P.info[j].state != SLOT_FREE) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0)
        P.ctl->done = (!any && P.ctl->next_job >= P.ctl->total_jobs) ? 1u : 0u;
}

struct ServerReq {
    int64_t id = 0;
    int32_t inst = 0, kind = 0, count = 0, njobs = 0;
    std::vector<int32_t> vars;
    std::vector<double> lb, ub;
    int32_t remaining = 0;
    bool on_device = false, done = false, cancelled = false;
    double submit_us = 0, done_us = 0;
    std::vector<JobOut> out;              // per job
    std::vector<std::vector<int32_t>> lvar; // per job implied lists
    std::vector<std::vector<double>> llb, lub;
};

// One slot pool: an engine whose slots hold any instance of its class, its
// job storage, launch parameters, captured rounds and stream.
struct ServerPool {
    Shape shape;                 // the slot shape (its class's largest instance)
    int32_t slots = 0;
    int64_t bytes_per_slot = 0;
    bool inc = false;            // incremental heavy rows over each instance's base
    int32_t members = 0;         // instances served by this pool
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::unique_ptr<Engine> eng;
    // device job storage
    DevBuf jobs, fix_var, fix_box, r_status, r_rounds, r_nnz, r_nbad, r_brow, r_bvar, r_soff, r_scnt;
    DevBuf stage_var, stage_lb, stage_ub, ring, collect;
    int64_t cap_jobs = 0, cap_fix = 0, cap_stage = 0;
    int64_t njobs_dev = 0, nfix_dev = 0;
    uint32_t ring_seen = 0;
    std::vector<int64_t> job_req;   // device job -> request id
    std::vector<int32_t> job_local; // device job -> index within its request
    std::deque<int64_t> pending;    // requests waiting for room in the job list
    Params P;
    JobIO IO;
    hipGraphExec_t graph = nullptr;
    int graph_rounds = 0;
    ~ServerPool() {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
};

struct bp_server {
    std::vector<bp_instance *> insts;  // nullptr: evicted
    std::vector<int64_t> inst_open;    // unfinished requests per instance
    std::vector<int32_t> inst_pool;    // pool of each instance
    int64_t cap_insts = 0;             // entries of the device instance table
    bp_options opt;
    int32_t heavy_chunk = 1024;
    hipStream_t st = nullptr;          // the caller's stream (the first pool's)
    DevBuf dinst;
    std::vector<std::unique_ptr<ServerPool>> pools;
    int64_t one_pool_bytes = 0;        // bytes of a slot sized for every instance
    // host side
    std::unordered_map<int64_t, ServerReq> reqs;
    std::deque<int64_t> completed;
    int64_t next_id = 1;
    int64_t unfinished = 0;
    std::vector<std::vector<uint8_t>> vtype;   // host copies for validation
    std::vector<std::vector<double2>> base;
    std::chrono::steady_clock::time_point t0;
    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Entries of a server's device instance table (instances added after
// creation take free entries; the table never moves, so captured graphs
// keep reading it).
constexpr int64_t SERVER_MAX_INSTANCES = 4096;
// Classes of instances, at most one stream each (the device's hardware
// queues run them side by side).
constexpr int SERVER_MAX_POOLS = 4;

// Device bytes one slot of shape `sh` needs (the engine's per-slot arrays;
// inc: with incremental heavy-row accumulators).
static int64_t slot_bytes(const Shape &sh, bool inc) {
    int64_t n = std::max<int64_t>(sh.sn, 1), m = std::max<int64_t>(sh.sm, 1);
    int64_t nw = (n + 31) / 32, mw = (m + 31) / 32;
    int64_t b = 16 * n + 16 * n + 8 * n + 4 * n;   // bounds, candidates, changed list, dirty list
    b += 4 * nw * 2 + 4 * mw;                      // var, dirty and row bitmaps
    b += 4 * FILT_WORDS + (int64_t)sizeof(SlotInfo) + 4;
    for (int q = 0; q < BIN_HEAVY; ++q) b += 2 * 8 * sh.bin_cap[q];
    b += 2 * 16 * sh.heavy_chunks + 64 * sh.heavy_chunks + 8 * sh.heavy_chunks;
    if (inc) b += sh.heavy_rows * (2 * HL * 8 + 8 + 8 + 16) + 2 * 16 * sh.heavy_chunks;
    return b;
}

static Shape shape_union(const Shape &a, const Shape &b) {
    Shape s;
    s.sn = std::max(a.sn, b.sn);
    s.sm = std::max(a.sm, b.sm);
    for (int q = 0; q < NBIN; ++q) s.bin_cap[q] = std::max(a.bin_cap[q], b.bin_cap[q]);
    s.heavy_chunks = std::max(a.heavy_chunks, b.heavy_chunks);
    s.heavy_rows = std::max(a.heavy_rows, b.heavy_rows);
    return s;
}

struct PoolPlan {
    std::vector<int32_t> members;
    Shape shape;
    bool inc = false;
    int64_t bytes = 0;
    int32_t slots = 0;
};

// Heavy rows of a pool keep exact corrections over their instance's base
// rows when every member keeps the limbs in range; otherwise (or with
// FULL_ROWS) they are summed chunk by chunk.
static void plan_finish(PoolPlan &p, const std::vector<bp_instance *> &insts, const bp_options &opt) {
    Shape sh;
    for (int32_t t : p.members) sh = shape_union(sh, shape_of(insts[t]));
    p.shape = sh;
    p.inc = sh.heavy_rows > 0 && !(opt.flags & BP_FLAG_FULL_ROWS);
    for (int32_t t : p.members) p.inc = p.inc && base_inc_ok(insts[t], opt.max_rounds);
    p.bytes = slot_bytes(sh, p.inc);
}

// The pools of a server.  Split: instances sorted by variables form classes
// of up to r times the class's smallest, r = max(8, (n_max / n_min)^(1/3.5)),
// so at most four.  The budget is shared out from the smallest slots up:
// each pool takes at most its fair share of what is left, and at most
// opt.probe_slots slots.
static std::vector<PoolPlan> plan_pools(const std::vector<bp_instance *> &insts, const bp_options &opt,
                                        int64_t budget, bool split) {
    std::vector<int32_t> order(insts.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return insts[a]->n < insts[b]->n; });
    std::vector<PoolPlan> plans;
    if (split) {
        const double nmin = std::max(1, insts[order.front()]->n), nmax = std::max(1, insts[order.back()]->n);
        const double r = std::max(8.0, std::pow(nmax / nmin, 1.0 / 3.5));
        for (int32_t t : order) {
            if (plans.empty() || (double)insts[t]->n > r * std::max(1, insts[plans.back().members[0]]->n))
                plans.emplace_back();
            plans.back().members.push_back(t);
        }
    } else {
        plans.emplace_back();
        plans.back().members = order;
    }
    for (PoolPlan &p : plans) plan_finish(p, insts, opt);
    std::stable_sort(plans.begin(), plans.end(), [](const PoolPlan &a, const PoolPlan &b) { return a.bytes < b.bytes; });
    const int64_t cap = std::max(1, opt.probe_slots);
    int64_t left = budget;
    for (size_t i = 0; i < plans.size(); ++i) {
        const int64_t share = left / (int64_t)(plans.size() - i);
        plans[i].slots = (int32_t)std::min<int64_t>(cap, share / plans[i].bytes);
        left -= (int64_t)plans[i].slots * plans[i].bytes;
    }
    return plans;
}

// Allocate a pool's engine and job storage and set its launch parameters.
static int pool_create(bp_server *sv, ServerPool &pl, const PoolPlan &plan, bool first) {
    pl.shape = plan.shape;
    pl.slots = plan.slots;
    pl.bytes_per_slot = plan.bytes;
    pl.inc = plan.inc;
    pl.members = (int32_t)plan.members.size();
    if (first) {
        pl.st = sv->st;
    } else {
        HIPTRY(hipStreamCreateWithFlags(&pl.st, hipStreamNonBlocking));
        pl.own_stream = true;
    }
    hipStream_t st = pl.st;
    if (int rc = engine_alloc(pl.eng, pl.shape, pl.slots, true, false, st, pl.inc)) return rc;
    int64_t dummy = 0;
    pl.cap_jobs = 1 << 21;
    pl.cap_fix = 1 << 24;
    pl.cap_stage = 1 << 25;
    const int64_t J = pl.cap_jobs;
    int rc;
    if ((rc = pl.jobs.alloc(J * sizeof(Job), dummy))) return rc;
    if ((rc = pl.fix_var.alloc(pl.cap_fix * 4, dummy))) return rc;
    if ((rc = pl.fix_box.alloc(pl.cap_fix * 16, dummy))) return rc;
    if ((rc = pl.r_status.alloc(J, dummy))) return rc;
    if ((rc = pl.r_rounds.alloc(J * 4, dummy))) return rc;
    if ((rc = pl.r_nnz.alloc(J * 8, dummy))) return rc;
    if ((rc = pl.r_nbad.alloc(J * 4, dummy))) return rc;
    if ((rc = pl.r_brow.alloc(J * 4, dummy))) return rc;
    if ((rc = pl.r_bvar.alloc(J * 4, dummy))) return rc;
    if ((rc = pl.r_soff.alloc(J * 8, dummy))) return rc;
    if ((rc = pl.r_scnt.alloc(J * 8, dummy))) return rc;
    if ((rc = pl.stage_var.alloc(pl.cap_stage * 4, dummy))) return rc;
    if ((rc = pl.stage_lb.alloc(pl.cap_stage * 8, dummy))) return rc;
    if ((rc = pl.stage_ub.alloc(pl.cap_stage * 8, dummy))) return rc;
    if ((rc = pl.ring.alloc(J * 4, dummy))) return rc;
    if ((rc = pl.collect.alloc(J * sizeof(JobOut), dummy))) return rc;
    JobIO &IO = pl.IO;
    memset(&IO, 0, sizeof(IO));
    IO.jobs = pl.jobs.as<Job>();
    IO.fix_var = pl.fix_var.as<int32_t>();
    IO.fix_box = pl.fix_box.as<double2>();
    IO.status = pl.r_status.as<int8_t>();
    IO.rounds = pl.r_rounds.as<int32_t>();
    IO.nnz = pl.r_nnz.as<int64_t>();
    IO.n_bad_rows = pl.r_nbad.as<int32_t>();
    IO.bad_row = pl.r_brow.as<int32_t>();
    IO.bad_var = pl.r_bvar.as<int32_t>();
    IO.stage_off = pl.r_soff.as<int64_t>();
    IO.stage_cnt = pl.r_scnt.as<int64_t>();
    IO.stage_var = pl.stage_var.as<int32_t>();
    IO.stage_lb = pl.stage_lb.as<double>();
    IO.stage_ub = pl.stage_ub.as<double>();
    IO.stage_cap = pl.cap_stage;
    IO.done_ring = pl.ring.as<uint32_t>();
    Params P = engine_params(*pl.eng, sv->opt, sv->heavy_chunk, pl.slots);
    P.I = dinst_of(sv->insts[plan.members[0]]);
    P.multi = 1;
    P.useen = nullptr;  // row ids repeat across instances
    P.insts = sv->dinst.as<DInst>();
    P.overlay = 1;
    if (pl.inc) {
        Engine &E = *pl.eng;
        P.inc = 1;
        P.nheavy = (int32_t)pl.shape.heavy_rows;
        P.inc_slots = pl.slots;
        P.hacc = E.hacc.as<long long>();
        P.hinf = E.hinf.as<int32_t>();
        P.hwid = E.hwid.as<unsigned long long>();
        P.hact = E.hact.as<double2>();
        P.hcrec[0] = E.hcrec[0].as<int4>();
        P.hcrec[1] = E.hcrec[1].as<int4>();
        P.inc_max = 0xffffffffu;  // never rebuilt
        P.inc_period = 0;
        P.inc_base = 1;
        // retired jobs clear their own corrections from here on
        HIPTRY(hipMemsetAsync(E.hacc.p, 0, (size_t)pl.slots * pl.shape.heavy_rows * 2 * HL * 8, st));
        HIPTRY(hipMemsetAsync(E.hinf.p, 0, (size_t)pl.slots * pl.shape.heavy_rows * 8, st));
    }
    pl.P = P;
    Ctl c;
    memset(&c, 0, sizeof(c));
    c.max_rounds = (uint32_t)sv->opt.max_rounds;
    c.nslots = (uint32_t)pl.slots;
    c.done = 1;
    HIPTRY(hipMemcpyAsync(P.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, st));
    k_reset_slots<<<grid_for(pl.slots), 256, 0, st>>>(P.info, pl.slots, 0, SLOT_FREE);
    HIPTRY(hipGetLastError());
    return 0;
}

extern "C" int bp_server_create(bp_instance *const *instances, int32_t count, const bp_options *opt,
                                int64_t budget_bytes, void *stream, bp_server **out) {
    BP_RANGE("bp_server_create");
    g_err.clear();
    if (!instances || count <= 0 || !out || budget_bytes <= 0)
        return fail(BP_EINVAL, "bp_server_create: bad argument");
    *out = nullptr;
    std::unique_ptr<bp_server> sv(new bp_server());
    sv->st = as_stream(stream);
    if (!opt && !instances[0]) return fail(BP_EINVAL, "bp_server_create: null instance");
    sv->opt = opt ? *opt : instances[0]->opt;
    if (int rc = validate_options(sv->opt)) return rc;
    if (sv->opt.rounds_per_launch <= 0) sv->opt.rounds_per_launch = 16;
    for (int32_t t = 0; t < count; ++t) {
        bp_instance *h = instances[t];
        if (!h) return fail(BP_EINVAL, "bp_server_create: null instance");
        BP_TABLES_CHECK(h);
        if (!h->have_base) return fail(BP_ESTATE, "instance " + std::to_string(t) + " has no base");
        if (t == 0) sv->heavy_chunk = h->heavy_chunk;
        else if (h->heavy_chunk != sv->heavy_chunk)
            return fail(BP_EINVAL, "instances must share the heavy chunk size");
        sv->insts.push_back(h);
    }
    sv->inst_open.assign(sv->insts.size(), 0);
    // Pools by class; when the budget leaves a class fewer than
    // min(16, probe_slots) slots, every instance shares one pool.
    std::vector<PoolPlan> plans = plan_pools(sv->insts, sv->opt, budget_bytes, true);
    const int32_t least = std::min(16, std::max(1, sv->opt.probe_slots));
    for (const PoolPlan &p : plans)
        if (plans.size() > 1 && p.slots < least) {
            plans = plan_pools(sv->insts, sv->opt, budget_bytes, false);
            break;
        }
    {
        PoolPlan all;
        all.members.resize(sv->insts.size());
        std::iota(all.members.begin(), all.members.end(), 0);
        plan_finish(all, sv->insts, sv->opt);
        sv->one_pool_bytes = all.bytes;
    }
    if (plans[0].slots < 1 || plans.back().slots < 1)
        return fail(BP_ENOMEM, "budget smaller than one slot (" + std::to_string(plans.back().bytes) + " bytes)");
    hipStream_t st = sv->st;
    // the heavy rows of the pools that keep them incrementally, then the
    // instance table and host copies for request validation
    sv->inst_pool.assign(sv->insts.size(), 0);
    for (size_t q = 0; q < plans.size(); ++q)
        for (int32_t t : plans[q].members) {
            sv->inst_pool[t] = (int32_t)q;
            if (plans[q].inc)
                if (int rc = base_limbs(sv->insts[t], st)) return rc;
        }
    std::vector<DInst> tab;
    for (bp_instance *h : sv->insts) {
        tab.push_back(dinst_of(h));
        std::vector<uint8_t> vt(h->n);
        std::vector<double2> bs(h->n);
        if (h->n) {
            HIPTRY(hipMemcpyAsync(vt.data(), h->vtype.p, h->n, hipMemcpyDeviceToHost, st));
            HIPTRY(hipMemcpyAsync(bs.data(), h->base.p, (size_t)h->n * 16, hipMemcpyDeviceToHost, st));
        }
        sv->vtype.push_back(std::move(vt));
        sv->base.push_back(std::move(bs));
    }
    int64_t dummy = 0;
    sv->cap_insts = std::max<int64_t>((int64_t)tab.size(), SERVER_MAX_INSTANCES);
    if (int rc = sv->dinst.alloc((size_t)sv->cap_insts * sizeof(DInst), dummy)) return rc;
    HIPTRY(hipMemcpyAsync(sv->dinst.p, tab.data(), tab.size() * sizeof(DInst), hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    for (size_t q = 0; q < plans.size(); ++q) {
        sv->pools.emplace_back(new ServerPool());
        if (int rc = pool_create(sv.get(), *sv->pools.back(), plans[q], q == 0)) return rc;
    }
    for (auto &pl : sv->pools) HIPTRY(hipStreamSynchronize(pl->st));
    sv->t0 = std::chrono::steady_clock::now();
    *out = sv.release();
    return BP_OK;
}

extern "C" void bp_server_destroy(bp_server *sv) { delete sv; }

extern "C" int bp_server_info(const bp_server *sv, int32_t *slots, int64_t *bytes_per_slot) {
    if (!sv) return fail(BP_EINVAL, "bp_server_info: null server");
    int32_t tot = 0;
    for (const auto &pl : sv->pools) tot += pl->slots;
    if (slots) *slots = tot;
    if (bytes_per_slot) *bytes_per_slot = sv->one_pool_bytes;
    return BP_OK;
}

extern "C" int bp_server_pool_info(const bp_server *sv, int32_t pool, int32_t *npools, int32_t *slots,
                                   int64_t *bytes_per_slot, int32_t *instances) {
    if (!sv) return fail(BP_EINVAL, "bp_server_pool_info: null server");
    if (npools) *npools = (int32_t)sv->pools.size();
    if (pool < 0 || pool >= (int32_t)sv->pools.size()) {
        if (slots || bytes_per_slot || instances) return fail(BP_EINVAL, "bp_server_pool_info: no such pool");
        return BP_OK;
    }
    const ServerPool &pl = *sv->pools[pool];
    if (slots) *slots = pl.slots;
    if (bytes_per_slot) *bytes_per_slot = pl.bytes_per_slot;
    if (instances) *instances = pl.members;
    return BP_OK;
}

extern "C" int bp_server_add_instance(bp_server *sv, bp_instance *h, int32_t *index) {
    BP_RANGE("bp_server_add_instance");
    g_err.clear();
    if (!sv || !h || !index) return fail(BP_EINVAL, "bp_server_add_instance: null argument");
    BP_TABLES_CHECK(h);
    if (!h->have_base) return fail(BP_ESTATE, "instance has no base");
    if (h->heavy_chunk != sv->heavy_chunk) return fail(BP_EINVAL, "instances must share the heavy chunk size");
    for (bp_instance *o : sv->insts)
        if (o == h) return fail(BP_EINVAL, "instance already served");
    // the pool with the smallest slots that hold it
    int32_t q = -1;
    for (size_t c = 0; c < sv->pools.size(); ++c) {
        const ServerPool &pl = *sv->pools[c];
        if (!pl.shape.covers(shape_of(h))) continue;
        if (pl.inc && !base_inc_ok(h, sv->opt.max_rounds)) continue;
        if (q < 0 || pl.bytes_per_slot < sv->pools[q]->bytes_per_slot) q = (int32_t)c;
    }
    if (q < 0) return fail(BP_ECAPACITY, "instance larger than the server's slots");
    int32_t t = 0;
    while (t < (int32_t)sv->insts.size() && sv->insts[t]) ++t;
    if (t >= sv->cap_insts) return fail(BP_ECAPACITY, "instance table full");
    hipStream_t st = sv->st;
    std::vector<uint8_t> vt(h->n);
    std::vector<double2> bs(h->n);
    if (h->n) {
        HIPTRY(hipMemcpyAsync(vt.data(), h->vtype.p, h->n, hipMemcpyDeviceToHost, st));
        HIPTRY(hipMemcpyAsync(bs.data(), h->base.p, (size_t)h->n * 16, hipMemcpyDeviceToHost, st));
    }
    if (sv->pools[q]->inc)
        if (int rc = base_limbs(h, st)) return rc;
    const DInst d = dinst_of(h);
    HIPTRY(hipMemcpyAsync(sv->dinst.as<DInst>() + t, &d, sizeof(DInst), hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    if (t == (int32_t)sv->insts.size()) {
        sv->insts.push_back(h);
        sv->inst_open.push_back(0);
        sv->inst_pool.push_back(q);
        sv->vtype.push_back(std::move(vt));
        sv->base.push_back(std::move(bs));
    } else {
        sv->insts[t] = h;
        sv->inst_open[t] = 0;
        sv->inst_pool[t] = q;
        sv->vtype[t] = std::move(vt);
        sv->base[t] = std::move(bs);
    }
    sv->pools[q]->members += 1;
    *index = t;
    return BP_OK;
}

extern "C" int bp_server_evict(bp_server *sv, int32_t index) {
    g_err.clear();
    if (!sv || index < 0 || index >= (int32_t)sv->insts.size() || !sv->insts[index])
        return fail(BP_EINVAL, "bp_server_evict: no such instance");
    if (sv->inst_open[index] > 0)
        return fail(BP_ESTATE, "instance " + std::to_string(index) + " has unfinished requests");
    sv->insts[index] = nullptr;
    sv->pools[sv->inst_pool[index]]->members -= 1;
    // The launch parameters name one instance as the default descriptor;
    // point them at a served one (the graphs are captured again) so nothing
    // refers to an instance its owner may now free.
    for (bp_instance *o : sv->insts) {
        if (!o) continue;
        for (auto &pl : sv->pools) {
            pl->P.I = dinst_of(o);
            if (pl->graph) {
                (void)hipGraphExecDestroy(pl->graph);
                pl->graph = nullptr;
            }
        }
        break;
    }
    sv->vtype[index].clear();
    sv->vtype[index].shrink_to_fit();
    sv->base[index].clear();
    sv->base[index].shrink_to_fit();
    return BP_OK;
}

extern "C" int bp_server_submit(bp_server *sv, const bp_request *req, int64_t *id) {
    g_err.clear();
    if (!sv || !req || !id) return fail(BP_EINVAL, "bp_server_submit: null argument");
    if (req->instance < 0 || req->instance >= (int32_t)sv->insts.size())
        return fail(BP_EINVAL, "bad instance index");
    if (req->kind != BP_REQ_PROBE && req->kind != BP_REQ_PROPAGATE) return fail(BP_EINVAL, "bad kind");
    if (req->count < 0 || (req->count > 0 && !req->vars)) return fail(BP_EINVAL, "bad variable list");
    if (req->kind == BP_REQ_PROPAGATE && req->count > 0 && (!req->lb || !req->ub))
        return fail(BP_EINVAL, "propagate request without bounds");
    const bp_instance *h = sv->insts[req->instance];
    if (!h) return fail(BP_EINVAL, "instance " + std::to_string(req->instance) + " was evicted");
    ServerPool &pl = *sv->pools[sv->inst_pool[req->instance]];
    const int64_t njobs = req->kind == BP_REQ_PROBE ? 2 * (int64_t)req->count : 1;
    if (njobs > pl.cap_jobs || (req->kind == BP_REQ_PROPAGATE && req->count > pl.cap_fix))
        return fail(BP_EINVAL, "request larger than the server's job storage");
    std::vector<int32_t> seen;
    seen.assign(req->vars, req->vars + req->count);
    std::sort(seen.begin(), seen.end());
    for (size_t t = 0; t < seen.size(); ++t) {
        if (seen[t] < 0 || seen[t] >= h->n) return fail(BP_EINVAL, "variable out of range");
        if (t && seen[t] == seen[t - 1]) return fail(BP_EINVAL, "repeated variable in a request");
    }
    if (req->kind == BP_REQ_PROBE) {
        for (int32_t t = 0; t < req->count; ++t) {
            int32_t j = req->vars[t];
            const double2 b = sv->base[req->instance][j];
            if (!sv->vtype[req->instance][j] || (std::isinf(b.x) && std::isinf(b.y)))
                return fail(BP_EINVAL, "probe variable is not an integer with a finite base bound");
        }
    } else {
        for (int32_t t = 0; t < req->count; ++t)
            if (std::isnan(req->lb[t]) || std::isnan(req->ub[t])) return fail(BP_EINVAL, "NaN bound");
    }
    ServerReq R;
    R.id = sv->next_id++;
    R.inst = req->instance;
    R.kind = req->kind;
    R.count = req->count;
    R.njobs = (int32_t)njobs;
    R.vars.assign(req->vars, req->vars + req->count);
    if (req->kind == BP_REQ_PROPAGATE) {
        R.lb.assign(req->lb, req->lb + req->count);
        R.ub.assign(req->ub, req->ub + req->count);
    }
    R.remaining = R.njobs;
    R.submit_us = sv->now_us();
    R.out.resize(R.njobs);
    R.lvar.resize(R.njobs);
    R.llb.resize(R.njobs);
    R.lub.resize(R.njobs);
    *id = R.id;
    if (R.njobs == 0) {  // nothing to run: finished at once
        R.done = true;
        R.done_us = R.submit_us;
        sv->completed.push_back(R.id);
        sv->reqs.emplace(R.id, std::move(R));
        return BP_OK;
    }
    pl.pending.push_back(R.id);
    sv->inst_open[R.inst] += 1;
    sv->reqs.emplace(R.id, std::move(R));
    sv->unfinished += 1;
    return BP_OK;
}

// Copy a pool's queued requests into its device job list while it has room.
static int server_append(bp_server *sv, ServerPool &pl) {
    hipStream_t st = pl.st;
    // The job list is rewound whenever every job on it has finished.
    if (pl.njobs_dev > 0 && pl.ring_seen == (uint32_t)pl.njobs_dev && !pl.pending.empty()) {
        pl.njobs_dev = 0;
        pl.nfix_dev = 0;
        pl.ring_seen = 0;
        pl.job_req.clear();
        pl.job_local.clear();
        uint32_t zeros[4] = {0, 0, 0, 0};
        Ctl *C = pl.P.ctl;
        HIPTRY(hipMemcpyAsync(&C->next_job, zeros, 12, hipMemcpyHostToDevice, st));  // next, total, done_jobs
        unsigned long long z = 0;
        HIPTRY(hipMemcpyAsync(&C->stage_count, &z, 8, hipMemcpyHostToDevice, st));
    }
    std::vector<Job> nj;
    std::vector<int32_t> fv;
    std::vector<double2> fb;
    while (!pl.pending.empty()) {
        ServerReq &R = sv->reqs[pl.pending.front()];
        int64_t nfix = R.kind == BP_REQ_PROPAGATE ? R.count : 0;
        if (pl.njobs_dev + (int64_t)nj.size() + R.njobs > pl.cap_jobs) break;
        if (pl.nfix_dev + (int64_t)fv.size() + nfix > pl.cap_fix) break;
        for (int32_t j = 0; j < R.njobs; ++j) {
            Job J;
            J.inst = R.inst;
            if (R.kind == BP_REQ_PROBE) {
                J.kind = JOB_PROBE;
                J.a = R.vars[j >> 1];
                J.b = j & 1;
            } else {
                J.kind = JOB_FIX;
                J.a = (int32_t)(pl.nfix_dev + (int64_t)fv.size());
                J.b = R.count;
                for (int32_t t = 0; t < R.count; ++t) {
                    fv.push_back(R.vars[t]);
                    fb.push_back(make_double2(R.lb[t], R.ub[t]));
                }
            }
            nj.push_back(J);
            pl.job_req.push_back(R.id);
            pl.job_local.push_back(j);
        }
        R.on_device = true;
        pl.pending.pop_front();
    }
    if (nj.empty()) return 0;
    // Claims past the end of the list took no job; lower the counter to the
    // old end so the appended jobs are claimed (the stream is idle here).
    {
        uint32_t next = 0;
        HIPTRY(hipMemcpyAsync(&next, &pl.P.ctl->next_job, 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (next > (uint32_t)pl.njobs_dev) {
            uint32_t old_end = (uint32_t)pl.njobs_dev;
            HIPTRY(hipMemcpyAsync(&pl.P.ctl->next_job, &old_end, 4, hipMemcpyHostToDevice, st));
        }
    }
    HIPTRY(hipMemcpyAsync(pl.jobs.as<Job>() + pl.njobs_dev, nj.data(), nj.size() * sizeof(Job),
                          hipMemcpyHostToDevice, st));
    if (!fv.empty()) {
        HIPTRY(hipMemcpyAsync(pl.fix_var.as<int32_t>() + pl.nfix_dev, fv.data(), fv.size() * 4,
                              hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(pl.fix_box.as<double2>() + pl.nfix_dev, fb.data(), fb.size() * 16,
                              hipMemcpyHostToDevice, st));
    }
    pl.njobs_dev += (int64_t)nj.size();
    pl.nfix_dev += (int64_t)fv.size();
    uint32_t tot = (uint32_t)pl.njobs_dev;
    HIPTRY(hipMemcpyAsync(&pl.P.ctl->total_jobs, &tot, 4, hipMemcpyHostToDevice, st));
    // the claims the last round end assigned predate these jobs
    const uint32_t no_claims = 0;
    HIPTRY(hipMemcpyAsync(&pl.P.ctl->claims, &no_claims, 4, hipMemcpyHostToDevice, st));
    // Admit right away, then recompute the done flag.
    k_retire<true><<<std::min(pl.slots, 4096), WG, 0, st>>>(pl.P, pl.IO);
    k_jobs_done_check<<<1, 256, 0, st>>>(pl.P);
    HIPTRY(hipGetLastError());
    return 0;
}

// Gather a pool's finished jobs from its completion ring and finish requests.
static int server_collect(bp_server *sv, ServerPool &pl) {
    hipStream_t st = pl.st;
    Ctl hc;
    HIPTRY(hipMemcpyAsync(&hc, pl.P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    const uint32_t r0 = pl.ring_seen, r1 = hc.done_jobs;
    if (r1 == r0) return 0;
    if (hc.stage_count > (unsigned long long)pl.cap_stage)
        return fail(BP_ECAPACITY, "server implication storage exceeded");
    const int64_t nr = r1 - r0;
    k_collect<<<grid_for(nr), 256, 0, st>>>(pl.IO, pl.ring.as<uint32_t>(), r0, r1, pl.collect.as<JobOut>());
    HIPTRY(hipGetLastError());
    std::vector<JobOut> got(nr);
    HIPTRY(hipMemcpyAsync(got.data(), pl.collect.p, nr * sizeof(JobOut), hipMemcpyDeviceToHost, st));
    // their lists form one contiguous range of the stage
    int64_t s0 = INT64_MAX, s1 = 0;
    HIPTRY(hipStreamSynchronize(st));
    for (const JobOut &o : got) {
        if (o.stage_cnt > 0) {
            s0 = std::min<int64_t>(s0, o.stage_off);
            s1 = std::max<int64_t>(s1, o.stage_off + o.stage_cnt);
        }
    }
    std::vector<int32_t> sv_var;
    std::vector<double> sv_lb, sv_ub;
    if (s1 > s0) {
        int64_t c = s1 - s0;
        sv_var.resize(c);
        sv_lb.resize(c);
        sv_ub.resize(c);
        HIPTRY(hipMemcpyAsync(sv_var.data(), pl.stage_var.as<int32_t>() + s0, c * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipMemcpyAsync(sv_lb.data(), pl.stage_lb.as<double>() + s0, c * 8, hipMemcpyDeviceToHost, st));
        HIPTRY(hipMemcpyAsync(sv_ub.data(), pl.stage_ub.as<double>() + s0, c * 8, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
    }
    const double t = sv->now_us();
    for (const JobOut &o : got) {
        ServerReq &R = sv->reqs[pl.job_req[o.job]];
        int32_t j = pl.job_local[o.job];
        R.out[j] = o;
        if (o.stage_cnt > 0) {
            int64_t a = o.stage_off - s0;
            R.lvar[j].assign(sv_var.begin() + a, sv_var.begin() + a + o.stage_cnt);
            R.llb[j].assign(sv_lb.begin() + a, sv_lb.begin() + a + o.stage_cnt);
            R.lub[j].assign(sv_ub.begin() + a, sv_ub.begin() + a + o.stage_cnt);
        }
        if (--R.remaining == 0) {
            R.done = true;
            R.done_us = t;
            sv->completed.push_back(R.id);
            sv->unfinished -= 1;
            sv->inst_open[R.inst] -= 1;
        }
    }
    pl.ring_seen = r1;
    return 0;
}

static int pool_graph(bp_server *sv, ServerPool &pl) {
    const int K = std::max(1, (int)sv->opt.rounds_per_launch);
    if (pl.graph && pl.graph_rounds == K) return 0;
    if (pl.graph) (void)hipGraphExecDestroy(pl.graph);
    pl.graph = nullptr;
    hipStream_t cs;
    HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < K; ++r) {
        k_rows<true><<<GRID_ROWS, WG, 0, cs>>>(pl.P);
        if (!pl.P.inc_base) k_heavy<true><<<GRID_HEAVY, WG, 0, cs>>>(pl.P);  // heavy rows decided by the heads
        k_apply<true><<<GRID_APPLY, WG, 0, cs>>>(pl.P);
        k_end<END_WG><<<1, END_WG, 0, cs>>>(pl.P);
        k_retire<true><<<std::min(pl.slots, 4096), WG, 0, cs>>>(pl.P, pl.IO);
    }
    hipGraph_t g;
    HIPTRY(hipStreamEndCapture(cs, &g));
    hipError_t e = hipGraphInstantiate(&pl.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    HIPTRY(e);
    pl.graph_rounds = K;
    return 0;
}

extern "C" int bp_server_run(bp_server *sv, int32_t rounds, int32_t *busy) {
    BP_RANGE("bp_server_run");
    g_err.clear();
    if (!sv || rounds < 0) return fail(BP_EINVAL, "bp_server_run: bad argument");
    hipStream_t st = sv->st;
    {
        // an instance whose base moved since its base rows were summed gets
        // them again (every pool's stream is idle between runs)
        bool moved = false;
        for (size_t t = 0; t < sv->insts.size(); ++t) {
            bp_instance *h = sv->insts[t];
            if (!h || !sv->pools[sv->inst_pool[t]]->inc || h->hb_version == h->base_version) continue;
            if (int rc = base_limbs(h, st)) return rc;
            const DInst d = dinst_of(h);
            HIPTRY(hipMemcpyAsync(sv->dinst.as<DInst>() + t, &d, sizeof(DInst), hipMemcpyHostToDevice, st));
            moved = true;
        }
        if (moved) HIPTRY(hipStreamSynchronize(st));
    }
    for (auto &pl : sv->pools) {
        if (int rc = server_append(sv, *pl)) return rc;
        if (int rc = pool_graph(sv, *pl)) return rc;
    }
    const int K = std::max(1, (int)sv->opt.rounds_per_launch);
    std::vector<char> live(sv->pools.size());
    for (int32_t r = 0; r < rounds; r += K) {
        // the pools with jobs on the device run side by side
        for (size_t q = 0; q < sv->pools.size(); ++q) {
            ServerPool &pl = *sv->pools[q];
            live[q] = pl.njobs_dev > (int64_t)pl.ring_seen;
            if (live[q]) HIPTRY(hipGraphLaunch(pl.graph, pl.st));
        }
        for (size_t q = 0; q < sv->pools.size(); ++q) {
            if (!live[q]) continue;
            if (int rc = server_collect(sv, *sv->pools[q])) return rc;
            if (int rc = server_append(sv, *sv->pools[q])) return rc;
        }
    }
    if (rounds == 0)
        for (auto &pl : sv->pools)
            if (int rc = server_collect(sv, *pl)) return rc;
    if (busy) *busy = (int32_t)sv->unfinished;
    return BP_OK;
}

// Take a request that still waits in its pool's host queue out of it; it
// finishes at once as cancelled.
static void server_cancel_pending(bp_server *sv, std::deque<int64_t> &q, std::deque<int64_t>::iterator at,
                                  double t) {
    ServerReq &R = sv->reqs[*at];
    R.cancelled = true;
    R.done = true;
    R.done_us = t;
    sv->completed.push_back(R.id);
    sv->unfinished -= 1;
    sv->inst_open[R.inst] -= 1;
    q.erase(at);
}

extern "C" int bp_server_cancel(bp_server *sv, int64_t id) {
    g_err.clear();
    if (!sv) return fail(BP_EINVAL, "bp_server_cancel: null server");
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(BP_EINVAL, "unknown request id");
    const ServerReq &R = it->second;
    if (R.done || R.on_device)
        return fail(BP_ESTATE, R.done ? "request has finished" : "request's jobs are on the device");
    std::deque<int64_t> &q = sv->pools[sv->inst_pool[R.inst]]->pending;
    auto at = std::find(q.begin(), q.end(), id);
    if (at == q.end()) return fail(BP_ESTATE, "request is not queued");
    server_cancel_pending(sv, q, at, sv->now_us());
    return BP_OK;
}

extern "C" int bp_server_expire(bp_server *sv, double max_wait_us, int32_t *n) {
    g_err.clear();
    if (!sv || !(max_wait_us >= 0.0)) return fail(BP_EINVAL, "bp_server_expire: bad argument");
    const double t = sv->now_us();
    int32_t k = 0;
    for (auto &pl : sv->pools) {
        std::deque<int64_t> &q = pl->pending;
        for (auto at = q.begin(); at != q.end();) {
            if (t - sv->reqs[*at].submit_us > max_wait_us) {
                const auto pos = at - q.begin();
                server_cancel_pending(sv, q, at, t);
                at = q.begin() + pos;
                ++k;
            } else {
                ++at;
            }
        }
    }
    if (n) *n = k;
    return BP_OK;
}

extern "C" int bp_server_poll(bp_server *sv, bp_completion *out, int32_t max, int32_t *n) {
    if (!sv || !n || max < 0 || (max > 0 && !out)) return fail(BP_EINVAL, "bp_server_poll: bad argument");
    int32_t k = 0;
    while (k < max && !sv->completed.empty()) {
        const ServerReq &R = sv->reqs[sv->completed.front()];
        bp_completion &c = out[k++];
        c.id = R.id;
        c.instance = R.inst;
        c.kind = R.kind;
        c.jobs = R.njobs;
        c.flags = R.cancelled ? BP_COMPLETION_CANCELLED : 0;
        c.submit_us = R.submit_us;
        c.done_us = R.done_us;
        sv->completed.pop_front();
    }
    *n = k;
    return BP_OK;
}

extern "C" int bp_server_results(bp_server *sv, int64_t id, int8_t *status, int32_t *rounds,
                                 int64_t *nnz, int32_t *n_bad_rows, int32_t *bad_row,
                                 int32_t *bad_var, int64_t *off, int32_t *var, double *lb,
                                 double *ub, int64_t cap, int64_t *required) {
    g_err.clear();
    if (!sv) return fail(BP_EINVAL, "bp_server_results: null server");
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return fail(BP_EINVAL, "unknown request id");
    const ServerReq &R = it->second;
    if (R.cancelled) return fail(BP_ECANCELED, "request was cancelled before it ran");
    if (!R.done) return fail(BP_ESTATE, "request has not finished");
    int64_t tot = 0;
    for (int32_t j = 0; j < R.njobs; ++j) tot += (int64_t)R.lvar[j].size();
    if (required) *required = tot;
    if (tot > cap) return fail(BP_ECAPACITY, "lists need " + std::to_string(tot) + " entries");
    int64_t pos = 0;
    for (int32_t j = 0; j < R.njobs; ++j) {
        const JobOut &o = R.out[j];
        if (status) status[j] = (int8_t)o.status;
        if (rounds) rounds[j] = o.rounds;
        if (nnz) nnz[j] = o.nnz;
        if (n_bad_rows) n_bad_rows[j] = o.n_bad_rows;
        if (bad_row) bad_row[j] = o.bad_row;
        if (bad_var) bad_var[j] = o.bad_var;
        if (off) off[j] = pos;
        for (size_t t = 0; t < R.lvar[j].size(); ++t, ++pos) {
            if (var) var[pos] = R.lvar[j][t];
            if (lb) lb[pos] = R.llb[j][t];
            if (ub) ub[pos] = R.lub[j][t];
        }
    }
    if (off) off[R.njobs] = pos;
    return BP_OK;
}
