// bp_tune.h -- schedule autotuner (part of bp_engine.hip's translation unit;
// see include/bp.h for the C ABI).
//
// The schedule knobs change how rows are mapped to workgroups and how many
// rounds a graph holds, never the arithmetic: every candidate must return
// the same outcome, rounds and propagated nonzeros, and the tuner checks
// that on every trial.  Candidates are timed on the caller's own workload.
#pragma once
#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>

static std::string tune_key(const bp_instance *h) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ') c = '_';
    // row-length histogram by powers of two: independent of the schedule
    std::vector<int64_t> hist(34, 0);
    for (int32_t L : h->row_len) {
        int b = 0;
        while ((1ll << b) < L) ++b;
        hist[b] += 1;
    }
    std::ostringstream os;
    os << arch << "/m" << h->m << "/n" << h->n << "/z" << h->nnz << "/h";
    for (size_t b = 0; b < hist.size(); ++b)
        if (hist[b]) os << b << ":" << hist[b] << ",";
    return os.str();
}

// Schedules the engine supports; a cache line outside them is ignored.
static bool tuning_valid(const bp_tuning &t) {
    return t.heavy_threshold >= 1024 && t.heavy_chunk >= WG && t.heavy_chunk % WG == 0 &&
           t.rounds_per_launch >= 1 && t.probe_slots >= 0;
}

static bool tune_lookup(const char *path, const std::string &key, bp_tuning *t) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        bp_tuning x;
        memset(&x, 0, sizeof(x));
        if (!(is >> k >> x.heavy_threshold >> x.heavy_chunk >> x.rounds_per_launch >> x.probe_slots >> x.ms))
            continue;
        if (k == key && tuning_valid(x)) {
            *t = x;
            found = true;  // the last entry for a key wins
        }
    }
    return found;
}

static void tune_store(const char *path, const std::string &key, const bp_tuning &t) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), t.heavy_threshold, t.heavy_chunk,
            t.rounds_per_launch, t.probe_slots, t.ms);
    fclose(f);
}

static int tune_apply(bp_instance *h, const bp_tuning &t, hipStream_t st) {
    if (!tuning_valid(t)) return fail(BP_EINVAL, "tuning outside the supported schedule range");
    h->opt.heavy_threshold = t.heavy_threshold;
    h->opt.heavy_chunk = t.heavy_chunk;
    h->opt.rounds_per_launch = t.rounds_per_launch;
    if (t.probe_slots > 0) h->opt.probe_slots = t.probe_slots;
    if (h->heavy_threshold != t.heavy_threshold || h->heavy_chunk != t.heavy_chunk) {
        h->heavy_threshold = t.heavy_threshold;
        h->heavy_chunk = t.heavy_chunk;
        return bin_rows(h, st);
    }
    return 0;
}

extern "C" int bp_autotune(bp_instance *h, const double *lb, const double *ub, const int32_t *vars,
                           int32_t k, const char *cache_path, bp_tuning *out, void *stream) {
    BP_RANGE("bp_autotune");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !out || (h->n > 0 && (!lb || !ub)) || k < 0 || (k > 0 && !vars))
        return fail(BP_EINVAL, "bp_autotune: bad argument");
    hipStream_t st = as_stream(stream);
    const std::string key = tune_key(h);
    bp_tuning best;
    memset(&best, 0, sizeof(best));
    if (tune_lookup(cache_path, key, &best)) {
        if (int rc = tune_apply(h, best, st)) return rc;
        best.trials = 0;
        best.from_cache = 1;
        *out = best;
        return BP_OK;
    }
    const int64_t n = h->n;
    DevBuf wl, wu;
    int64_t dummy = 0;
    if (int rc = wl.alloc((size_t)std::max<int64_t>(n, 1) * 8, dummy)) return rc;
    if (int rc = wu.alloc((size_t)std::max<int64_t>(n, 1) * 8, dummy)) return rc;
    bp_result ref;
    bool have_ref = false;
    int trials = 0;
    // One timed cold propagation (best of two); checks the result is the
    // same for every schedule.
    auto time_prop = [&](double &ms) -> int {
        ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            if (n) {
                HIPTRY(hipMemcpyAsync(wl.p, lb, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
                HIPTRY(hipMemcpyAsync(wu.p, ub, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
            }
            HIPTRY(hipStreamSynchronize(st));
            bp_result r;
            auto t0 = std::chrono::steady_clock::now();
            int rc = bp_propagate(h, wl.as<double>(), wu.as<double>(), nullptr, 0, &r, st);
            auto t1 = std::chrono::steady_clock::now();
            if (rc < 0) return rc;
            ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
            if (!have_ref) {
                ref = r;
                have_ref = true;
            } else if (r.status != ref.status || r.rounds != ref.rounds ||
                       r.nnz_propagated != ref.nnz_propagated) {
                return fail(BP_EDEVICE, "autotuner: a schedule changed the propagation result");
            }
        }
        ++trials;
        return 0;
    };
    const int32_t thresholds[] = {2048, 4096, 8192, 16384, 32768};
    const int32_t chunks[] = {512, 1024, 2048, 4096};
    const int32_t rounds[] = {4, 8, 16, 32};
    best.ms = 1e300;
    bp_tuning cur = best;
    cur.rounds_per_launch = 16;
    cur.probe_slots = h->opt.probe_slots;
    for (int32_t ht : thresholds) {
        for (int32_t hc : chunks) {
            if (hc > ht) continue;
            cur.heavy_threshold = ht;
            cur.heavy_chunk = hc;
            if (int rc = tune_apply(h, cur, st)) return rc;
            double ms;
            if (int rc = time_prop(ms)) return rc;
            if (ms < best.ms) {
                best = cur;
                best.ms = ms;
            }
        }
    }
    for (int32_t rpl : rounds) {
        cur = best;
        cur.rounds_per_launch = rpl;
        if (int rc = tune_apply(h, cur, st)) return rc;
        double ms;
        if (int rc = time_prop(ms)) return rc;
        if (ms < best.ms) {
            best = cur;
            best.ms = ms;
        }
    }
    if (int rc = tune_apply(h, best, st)) return rc;
    double ms_final;
    if (int rc = time_prop(ms_final)) return rc;  // leaves the base at the cold result
    if (k > 0 && ref.status == BP_OK) {
        // Probe slots, timed on bp_probe of the caller's variables.
        const int64_t jobs = 2 * (int64_t)k;
        DevBuf ps, pr, pn, po;
        if (int rc = ps.alloc(jobs, dummy)) return rc;
        if (int rc = pr.alloc(jobs * 4, dummy)) return rc;
        if (int rc = pn.alloc(jobs * 8, dummy)) return rc;
        if (int rc = po.alloc((jobs + 1) * 8, dummy)) return rc;
        bp_probe_out o;
        memset(&o, 0, sizeof(o));
        o.status = ps.as<int8_t>();
        o.rounds = pr.as<int32_t>();
        o.nnz = pn.as<int64_t>();
        o.off = po.as<int64_t>();
        o.cap = 0;
        int rc = bp_probe(h, vars, k, &o, st);
        if (rc < 0 && rc != BP_ECAPACITY) return rc;
        const int64_t cap = std::max<int64_t>(o.required, 1);
        DevBuf pv, pl, pu;
        if ((rc = pv.alloc(cap * 4, dummy))) return rc;
        if ((rc = pl.alloc(cap * 8, dummy))) return rc;
        if ((rc = pu.alloc(cap * 8, dummy))) return rc;
        o.var = pv.as<int32_t>();
        o.lb = pl.as<double>();
        o.ub = pu.as<double>();
        o.cap = cap;
        const int32_t slot_opts[] = {64, 128, 256, 512, 1024, 2048};
        double best_probe = 1e300;
        int32_t best_slots = h->opt.probe_slots;
        for (int32_t sl : slot_opts) {
            if (sl > jobs && sl != slot_opts[0]) break;
            h->opt.probe_slots = sl;
            if ((rc = bp_probe(h, vars, k, &o, st)) < 0) return rc;  // warm (sizes the slots)
            auto t0 = std::chrono::steady_clock::now();
            if ((rc = bp_probe(h, vars, k, &o, st)) < 0) return rc;
            double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            ++trials;
            if (o.required != cap) return fail(BP_EDEVICE, "autotuner: a schedule changed the probe result");
            if (ms < best_probe) {
                best_probe = ms;
                best_slots = sl;
            }
        }
        h->opt.probe_slots = best_slots;
        best.probe_slots = best_slots;
    }
    best.trials = trials;
    best.from_cache = 0;
    tune_store(cache_path, key, best);
    *out = best;
    return BP_OK;
}

// ---------------------------------------------------------------------------
// Batched propagation: the lane engine's workgroups per round kernel and the
// rounds per graph, timed on the caller's batch (best of two calls each).
// ---------------------------------------------------------------------------
static bool tune_lookup_batch(const char *path, const std::string &key, bp_tuning *t) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        bp_tuning x;
        memset(&x, 0, sizeof(x));
        if (!(is >> k >> x.lv_grid >> x.rounds_per_launch >> x.ms)) continue;
        if (k == key && x.lv_grid >= 64 && x.rounds_per_launch >= 1) {
            *t = x;
            found = true;
        }
    }
    return found;
}

extern "C" int bp_autotune_batch(bp_instance *h, int32_t B, const double *lb, const double *ub,
                                 const int64_t *changed_ptr, const int32_t *changed_idx,
                                 const char *cache_path, bp_tuning *out, void *stream) {
    BP_RANGE("bp_autotune_batch");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !out || B <= 0 || (h->n > 0 && (!lb || !ub)))
        return fail(BP_EINVAL, "bp_autotune_batch: bad argument");
    hipStream_t st = as_stream(stream);
    std::ostringstream ks;
    ks << "batch/" << tune_key(h) << "/B" << B << (changed_ptr ? "/warm" : "/cold");
    const std::string key = ks.str();
    bp_tuning best;
    memset(&best, 0, sizeof(best));
    best.heavy_threshold = h->opt.heavy_threshold;
    best.heavy_chunk = h->opt.heavy_chunk;
    best.probe_slots = h->opt.probe_slots;
    if (tune_lookup_batch(cache_path, key, &best)) {
        h->opt.lv_grid = best.lv_grid;
        h->opt.rounds_per_launch = best.rounds_per_launch;
        best.heavy_threshold = h->opt.heavy_threshold;
        best.heavy_chunk = h->opt.heavy_chunk;
        best.probe_slots = h->opt.probe_slots;
        best.trials = 0;
        best.from_cache = 1;
        *out = best;
        return BP_OK;
    }
    const size_t N = (size_t)B * (size_t)std::max<int32_t>(h->n, 1);
    DevBuf wl, wu;
    int64_t dummy = 0;
    if (int rc = wl.alloc(N * 8, dummy)) return rc;
    if (int rc = wu.alloc(N * 8, dummy)) return rc;
    std::vector<bp_result> ref((size_t)B), res((size_t)B);
    bool have_ref = false;
    int trials = 0;
    auto time_batch = [&](double &ms) -> int {
        ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            if (h->n) {
                HIPTRY(hipMemcpyAsync(wl.p, lb, N * 8, hipMemcpyDeviceToDevice, st));
                HIPTRY(hipMemcpyAsync(wu.p, ub, N * 8, hipMemcpyDeviceToDevice, st));
            }
            HIPTRY(hipStreamSynchronize(st));
            auto t0 = std::chrono::steady_clock::now();
            int rc = bp_propagate_batch(h, B, wl.as<double>(), wu.as<double>(), changed_ptr, changed_idx,
                                        res.data(), st);
            auto t1 = std::chrono::steady_clock::now();
            if (rc < 0) return rc;
            ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
            if (!have_ref) {
                ref = res;
                have_ref = true;
            } else {
                for (int32_t j = 0; j < B; ++j)
                    if (res[j].status != ref[j].status || res[j].rounds != ref[j].rounds ||
                        res[j].nnz_propagated != ref[j].nnz_propagated)
                        return fail(BP_EDEVICE, "autotuner: a schedule changed a batch result");
            }
        }
        ++trials;
        return 0;
    };
    const int32_t grids[] = {1024, 2048, 4096, 8192};
    const int32_t rounds[] = {8, 16, 32};
    best.ms = 1e300;
    const int32_t saved_grid = h->opt.lv_grid, saved_rounds = h->opt.rounds_per_launch;
    int rc = 0;
    for (int32_t g : grids) {
        h->opt.lv_grid = g;
        h->opt.rounds_per_launch = 16;
        double ms;
        if ((rc = time_batch(ms))) break;
        if (ms < best.ms) {
            best.ms = ms;
            best.lv_grid = g;
            best.rounds_per_launch = 16;
        }
    }
    for (int32_t r : rounds) {
        if (rc) break;
        h->opt.lv_grid = best.lv_grid;
        h->opt.rounds_per_launch = r;
        double ms;
        if ((rc = time_batch(ms))) break;
        if (ms < best.ms) {
            best.ms = ms;
            best.rounds_per_launch = r;
        }
    }
    if (rc) {
        h->opt.lv_grid = saved_grid;
        h->opt.rounds_per_launch = saved_rounds;
        return rc;
    }
    h->opt.lv_grid = best.lv_grid;
    h->opt.rounds_per_launch = best.rounds_per_launch;
    best.trials = trials;
    best.from_cache = 0;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d %.6f\n", key.c_str(), best.lv_grid, best.rounds_per_launch, best.ms);
            fclose(f);
        }
    }
    *out = best;
    return BP_OK;
}

