// bp_lv_run.h -- host driver of the one-vector-per-lane batch engine (part
// of bp_engine.hip's translation unit; see bp_lv.h for the kernels).
#pragma once

#ifndef BP_LV_GRID
#define BP_LV_GRID 2048
#endif
static const int LV_GRID_ROWS = BP_LV_GRID;  // workgroups per round kernel, over all groups
static const int LV_MIN_BATCH = 16;     // smaller batches run on the slot engine

// Cold-start task tables of the instance: short rows, and (row, chunk) of
// the long rows.  They set the chunk-task capacity of a group.
static int lv_tables(bp_instance *h, LvEngine &L, hipStream_t st) {
    std::vector<int32_t> sr;
    std::vector<int2> lc;
    std::vector<int32_t> c0((size_t)std::max<int64_t>(h->m, 1), -1);  // chunk id of a long row's chunk 0
    for (int64_t k = 0; k < h->m; ++k) {
        const int64_t len = h->row_len[k];
        if (len <= LV_SHORT) {
            sr.push_back((int32_t)k);
        } else {
            const int64_t nch = (len + LV_CHUNK - 1) / LV_CHUNK;
            c0[k] = (int32_t)lc.size();
            for (int64_t c = 0; c < nch; ++c) lc.push_back(make_int2((int)k, (int)c));
        }
    }
    L.nshort = (int64_t)sr.size();
    L.nlong = (int64_t)lc.size();
    L.lcap = std::max<int64_t>(L.nlong, 1);
    int rc;
    if ((rc = L.short_rows.alloc(sr.size() * 4, h->bytes))) return rc;
    if ((rc = L.long_chunks.alloc(lc.size() * sizeof(int2), h->bytes))) return rc;
    if ((rc = L.lchunk0.alloc(c0.size() * 4, h->bytes))) return rc;
    HIPTRY(hipMemcpyAsync(L.lchunk0.p, c0.data(), c0.size() * 4, hipMemcpyHostToDevice, st));
    if (!sr.empty()) HIPTRY(hipMemcpyAsync(L.short_rows.p, sr.data(), sr.size() * 4, hipMemcpyHostToDevice, st));
    if (!lc.empty())
        HIPTRY(hipMemcpyAsync(L.long_chunks.p, lc.data(), lc.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    return 0;
}

// Buffers for V lanes (grow only).  The candidate keys are filled with
// (-inf, +inf) and every mask with zero once; each call leaves them so.
static int lv_ensure(bp_instance *h, int32_t V, bool count, hipStream_t st) {
    if (!h->lv) {
        // the engine is kept only once its tables exist
        std::unique_ptr<LvEngine> E(new LvEngine());
        if (int rc = lv_tables(h, *E, st)) {
            h->bytes -= (int64_t)(E->short_rows.bytes + E->long_chunks.bytes + E->lchunk0.bytes);
            return rc;
        }
        h->lv = std::move(E);
    }
    LvEngine &L = *h->lv;
    const int64_t n = std::max<int32_t>(h->n, 1), m = std::max<int32_t>(h->m, 1);
    int64_t &B = h->bytes;
    int rc;
    if (L.Vcap < V) {
        if (L.graph) {
            (void)hipGraphExecDestroy(L.graph);
            L.graph = nullptr;
        }
        const int64_t NG = V / 64;
        // Until every buffer below exists no call may use the old ones (a
        // failed allocation has already freed its buffer).
        L.Vcap = 0;
        L.have_touched = false;
        if ((rc = L.bnd.alloc((size_t)n * V * 16, B))) return rc;
        if ((rc = L.cand.alloc((size_t)n * V * 16, B))) return rc;
        if ((rc = L.vmask.alloc((size_t)NG * n * 8, B))) return rc;
        if ((rc = L.dmask.alloc((size_t)NG * n * 8, B))) return rc;
        for (int p = 0; p < 2; ++p) {
            if ((rc = L.rmask[p].alloc((size_t)NG * m * 8, B))) return rc;
            if ((rc = L.qs[p].alloc((size_t)NG * m * 4, B))) return rc;
            if ((rc = L.ql[p].alloc((size_t)NG * L.lcap * sizeof(int2), B))) return rc;
        }
        if ((rc = L.lpart.alloc((size_t)NG * L.lcap * 128 * sizeof(Acc), B))) return rc;
        if ((rc = L.lrng.alloc((size_t)NG * L.lcap * 64 * 8, B))) return rc;
        if ((rc = L.lmask.alloc((size_t)NG * L.lcap * 8, B))) return rc;
        if ((rc = L.chg.alloc((size_t)NG * n * 4, B))) return rc;
        if ((rc = L.vec.alloc((size_t)V * sizeof(LvVec), B))) return rc;
        if ((rc = L.vbad.alloc((size_t)V * 4, B))) return rc;
        if ((rc = L.wmask.alloc((size_t)V, B))) return rc;
        if ((rc = L.box.alloc((size_t)V * 8, B))) return rc;
        if (!L.ctl.p && (rc = L.ctl.alloc(sizeof(LvCtl), B))) return rc;
        k_lv_fill_cand<<<4096, 256, 0, st>>>(L.cand.as<longlong2>(), (size_t)n * V);
        k_lv_fill_u64<<<4096, 256, 0, st>>>(L.vmask.as<uint64_t>(), (size_t)NG * n);
        for (int p = 0; p < 2; ++p) k_lv_fill_u64<<<4096, 256, 0, st>>>(L.rmask[p].as<uint64_t>(), (size_t)NG * m);
        HIPTRY(hipGetLastError());
        L.Vcap = V;
        L.have_touched = false;
    }
    if (count && !L.have_touched) {
        const int64_t NG = L.Vcap / 64;
        if ((rc = L.touched.alloc((size_t)NG * n * 8, B))) return rc;
        if ((rc = L.rtouch.alloc((size_t)(m + 63) / 64 * 8, B))) return rc;
        k_lv_fill_u64<<<4096, 256, 0, st>>>(L.touched.as<uint64_t>(), (size_t)NG * n);
        k_lv_fill_u64<<<64, 256, 0, st>>>(L.rtouch.as<uint64_t>(), (size_t)(m + 63) / 64);
        HIPTRY(hipGetLastError());
        L.have_touched = true;
    }
    HIPTRY(hipStreamSynchronize(st));
    return 0;
}

// The long-row chunks at the base bounds (overlay mode), once per base.
static int lv_base_chunks(bp_instance *h, hipStream_t st) {
    LvEngine &L = *h->lv;
    if (L.nlong == 0 || L.lb_version == h->base_version) return 0;
    L.lb_version = -1;
    if (int rc = L.lbase.grow((size_t)L.nlong * 2 * sizeof(Acc), h->bytes)) return rc;
    if (int rc = L.lbw.grow((size_t)L.nlong * 8, h->bytes)) return rc;
    k_lv_base_chunks<<<(int)std::min<int64_t>((L.nlong + 3) / 4, 8192), WG, 0, st>>>(
        dinst_of(h), L.long_chunks.as<int2>(), L.nlong, L.lbase.as<Acc>(), L.lbw.as<double>());
    HIPTRY(hipGetLastError());
    L.lb_version = h->base_version;
    return 0;
}

// corr: long-row chunks may be summed as base plus corrections (each chunk
// task still decides from its own changed nonzeros).
static LvParams lv_params(const bp_instance *h, int32_t Bp, int32_t V, bool count, bool overlay,
                          bool corr = true) {
    LvEngine &L = *h->lv;
    LvParams P;
    memset(&P, 0, sizeof(P));
    P.I = dinst_of(h);
    P.feastol = h->opt.feastol;
    P.inttol = h->opt.inttol;
    P.tau = h->opt.tau;
    P.force_exact = (h->opt.flags & BP_FLAG_FORCE_EXACT) ? 1 : 0;
    P.count_vars = count ? 1 : 0;
    P.max_rounds = h->opt.max_rounds;
    P.B = Bp;
    P.V = V;
    P.NG = V / 64;
    P.m = h->m;
    P.n = h->n;
    P.bnd = L.bnd.as<double2>();
    P.base = overlay ? h->base.as<double2>() : nullptr;
    P.dmask = L.dmask.as<uint64_t>();
    P.cand = L.cand.as<longlong2>();
    P.vmask = L.vmask.as<uint64_t>();
    for (int p = 0; p < 2; ++p) {
        P.rmask[p] = L.rmask[p].as<uint64_t>();
        P.qs[p] = L.qs[p].as<int32_t>();
        P.ql[p] = L.ql[p].as<int2>();
    }
    P.lcap = L.lcap;
    P.lpart = L.lpart.as<Acc>();
    P.lrng = L.lrng.as<double>();
    P.lmask = L.lmask.as<uint64_t>();
    P.chg = L.chg.as<int32_t>();
    P.touched = count ? L.touched.as<uint64_t>() : nullptr;
    P.rtouch = count ? L.rtouch.as<uint32_t>() : nullptr;
    P.vec = L.vec.as<LvVec>();
    P.vbad = L.vbad.as<uint32_t>();
    P.ctl = L.ctl.as<LvCtl>();
    if (overlay && corr && L.nlong > 0 && L.lb_version == h->base_version) {
        P.lchunk0 = L.lchunk0.as<int32_t>();
        P.lbase = L.lbase.as<Acc>();
        P.lbw = L.lbw.as<double>();
    }
    return P;
}

// Workgroups of a lane round kernel over all groups: the instance's
// lv_grid option (the autotuner's choice), else LV_GRID_ROWS.
static int lv_grid(const bp_instance *h) { return h->opt.lv_grid > 0 ? h->opt.lv_grid : LV_GRID_ROWS; }

static void lv_launch_round(bp_instance *h, const LvParams &P, hipStream_t st, bool timed) {
    const int gx = std::max(1, lv_grid(h) / P.NG);
    const dim3 grid(gx, P.NG);
    if (timed) hipExtLaunchKernelGGL(k_lv_rows, grid, dim3(WG), 0, st, h->ev0, h->ev1, 0, P);
    else k_lv_rows<<<grid, WG, 0, st>>>(P);
    k_lv_heavy<<<grid, WG, 0, st>>>(P);
    k_lv_apply<<<dim3(std::max(1, GRID_APPLY * 2 / P.NG), P.NG), WG, 0, st>>>(P, 0);
    k_lv_end<<<1, WG, 0, st>>>(P);
}

// Rounds until every vector is finished: graphs of K rounds, or host rounds
// with the row kernel timed by events.
static int lv_run_rounds(bp_instance *h, const LvParams &P, hipStream_t st) {
    LvEngine &L = *h->lv;
    const bool timed = (h->opt.flags & BP_FLAG_TIME_KERNELS) != 0;
    const bool host_rounds = timed || (h->opt.flags & BP_FLAG_HOST_ROUNDS) != 0;
    const int K = std::max(1, (int)h->opt.rounds_per_launch);
    const int64_t limit = (int64_t)h->opt.max_rounds + 2;
    if (L.graph && (L.graph_rounds != K || memcmp(&L.graph_params, &P, sizeof(LvParams)) != 0)) {
        (void)hipGraphExecDestroy(L.graph);
        L.graph = nullptr;
    }
    LvCtl hc;
    int64_t launched = 0;
    for (;;) {
        if (host_rounds) {
            lv_launch_round(h, P, st, timed);
            HIPTRY(hipGetLastError());
            launched += 1;
            if (timed) {
                HIPTRY(hipEventSynchronize(h->ev1));
                float ms = 0.f;
                HIPTRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
                h->stats.ms += ms;
                h->stats.launches += 1;
            }
        } else {
            if (!L.graph) {
                hipStream_t cs;
                HIPTRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                for (int r = 0; r < K; ++r) lv_launch_round(h, P, cs, false);
                hipGraph_t g;
                HIPTRY(hipStreamEndCapture(cs, &g));
                hipError_t e = hipGraphInstantiate(&L.graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                (void)hipStreamDestroy(cs);
                HIPTRY(e);
                L.graph_rounds = K;
                L.graph_params = P;
            }
            HIPTRY(hipGraphLaunch(L.graph, st));
            launched += K;
        }
        HIPTRY(hipMemcpyAsync(&hc, P.ctl, sizeof(LvCtl), hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (hc.done) break;
        if (launched > limit) return fail(BP_EDEVICE, "round loop did not terminate");
    }
    h->stats.rows += (int64_t)hc.stat_rows;
    h->stats.nnz += (int64_t)hc.stat_nnz;
    h->stats.vars_read += (int64_t)hc.stat_vars;
    h->stats.vars_written += (int64_t)hc.stat_written;
    h->stats.lv_corr_chunks += (int64_t)hc.stat_corr;
    return 0;
}

static void lv_fill_result(const LvVec &S, int32_t box_bad, bp_result *r) {
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
    r->nnz_propagated = (int64_t)S.nnz;
    if (S.status == BP_INFEASIBLE) {
        if (S.row_bad_count > 0) {
            r->n_infeasible_rows = S.row_bad_count;
            r->infeasible_row = S.row_bad_min;
        } else {
            r->infeasible_var = S.var_bad_min;
        }
    }
}

// One piece of a batch: vectors [0, Bp) of lb/ub (row-major [Bp][n]), their
// changed lists given by ptr (absolute offsets into idx, Bp + 1 entries).
static int lv_piece(bp_instance *h, int32_t Bp, double *lb, double *ub, const int32_t *idx,
                    const int64_t *ptr_dev, int64_t e0, int64_t ecount, bool cold, bp_result *res,
                    hipStream_t st) {
    const int32_t V = (Bp + 63) / 64 * 64;
    const bool count = (h->opt.flags & BP_FLAG_COUNT_VARS) != 0;
    if (int rc = lv_ensure(h, V, count, st)) return rc;
    LvEngine &L = *h->lv;
    // Overlay mode when the instance has a base box (bulk-rounding
    // candidates are the base with a few fixings); results are identical.
    const bool overlay = h->have_base && !(h->opt.flags & BP_FLAG_LV_DENSE);
    if (overlay)
        if (int rc = lv_base_chunks(h, st)) return rc;
    // A batch whose vectors change more than n/96 variables each on average
    // leaves most of a 64-vector group's nonzeros changed in some lane
    // (1 - (1 - 1/96)^64 > 1/2): its chunks are summed whole without the
    // per-chunk test.
    const bool corr = cold || ecount * 96 <= (int64_t)Bp * h->n;
    const LvParams P = lv_params(h, Bp, V, count, overlay, corr);
    const int64_t n = h->n;
    const int NG = P.NG;
    // bounds in, box check
    {
        std::vector<int32_t> init(2 * (size_t)V);
        for (int32_t j = 0; j < V; ++j) {
            init[2 * j] = NONE;
            init[2 * j + 1] = 0;
        }
        HIPTRY(hipMemcpyAsync(L.box.p, init.data(), init.size() * 4, hipMemcpyHostToDevice, st));
    }
    if (n > 0) {
        const int64_t tiles = (n + 63) / 64 * NG;
        if (P.base)
            k_lv_pack_overlay<<<(int)std::min<int64_t>(tiles, 16384), WG, 0, st>>>(
                lb, ub, P.bnd, (int32_t)n, Bp, V, h->vtype.as<uint8_t>(), h->opt.feastol, L.box.as<int32_t>(),
                P.base, P.dmask);
        else
            k_lv_pack<<<(int)std::min<int64_t>(tiles, 8192), WG, 0, st>>>(lb, ub, P.bnd, (int32_t)n, Bp, V,
                                                                         h->vtype.as<uint8_t>(), h->opt.feastol,
                                                                         L.box.as<int32_t>(), P.base, P.dmask);
    }
    HIPTRY(hipGetLastError());
    std::vector<int32_t> box(2 * (size_t)V);
    HIPTRY(hipMemcpyAsync(box.data(), L.box.p, box.size() * 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    for (int32_t j = 0; j < Bp; ++j)
        if (box[2 * j + 1]) return fail(BP_EINVAL, "NaN bound in vector " + std::to_string(j));
    if (!cold && ecount > 0)
        if (int rc = check_ids(h, idx + e0, ecount, st)) return rc;
    // control block, vectors, seeds
    LvCtl c;
    memset(&c, 0, sizeof(c));
    HIPTRY(hipMemcpyAsync(P.ctl, &c, sizeof(LvCtl), hipMemcpyHostToDevice, st));
    k_lv_reset<<<grid_for(V), 256, 0, st>>>(P, L.box.as<int32_t>());
    const int gx = std::max(1, lv_grid(h) / NG);
    if (cold) {
        if (h->m > 0)
            k_lv_seed_cold<<<dim3(std::max(1, gx / 4), NG), 256, 0, st>>>(
                P, L.short_rows.as<int32_t>(), L.nshort, L.long_chunks.as<int2>(), L.nlong);
    } else if (ecount > 0) {
        // Queue the rows of the listed variables: by columns (one atomic per
        // column entry and group) for short lists, by rows (a read of the
        // matrix per group, no atomics) when the columns would cover a good
        // part of it.  The row path needs only the (group, variable) masks,
        // which it then clears whole.
        const double col_cost = 4.0 * (double)std::min<int64_t>(ecount, (int64_t)n * NG) *
                                ((double)h->nnz / (double)std::max<int64_t>(n, 1));
        const double row_cost = (double)NG * ((double)h->nnz + (double)h->m);
        const bool by_rows = col_cost > row_cost;
        k_lv_seed_vars<<<grid_for(ecount), 256, 0, st>>>(P, idx, ptr_dev, e0, ecount, by_rows ? 0 : 1);
        if (by_rows) {
            k_lv_seed_rows<<<dim3(gx, NG), WG, 0, st>>>(P);
            k_lv_fill_u64<<<4096, 256, 0, st>>>(P.vmask, (size_t)NG * n);
        } else {
            k_lv_apply<<<dim3(gx, NG), WG, 0, st>>>(P, 1);
        }
    }
    k_lv_seed_finish<<<grid_for(V), 256, 0, st>>>(P, cold ? 1 : 0, (long long)h->nnz);
    k_lv_start<<<1, 256, 0, st>>>(P);
    HIPTRY(hipGetLastError());
    if (int rc = lv_run_rounds(h, P, st)) return rc;
    k_lv_cleanup<<<dim3(std::max(1, gx / 4), NG), 256, 0, st>>>(P);
    k_lv_cleanup_counts<<<1, 64, 0, st>>>(P);
    HIPTRY(hipGetLastError());
    std::vector<LvVec> vec(Bp);
    HIPTRY(hipMemcpyAsync(vec.data(), P.vec, Bp * sizeof(LvVec), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    for (int32_t j = 0; j < Bp; ++j) lv_fill_result(vec[j], box[2 * j], &res[j]);
    // Bounds out, except for infeasible vectors (their bounds are
    // unspecified; they keep the input).
    std::vector<uint8_t> wm(V, 0);
    bool any = false;
    for (int32_t j = 0; j < Bp; ++j) {
        wm[j] = res[j].status != BP_INFEASIBLE;
        any = any || wm[j];
    }
    if (n > 0 && any) {
        HIPTRY(hipMemcpyAsync(L.wmask.p, wm.data(), V, hipMemcpyHostToDevice, st));
        const int64_t tiles = (n + 63) / 64 * NG;
        k_lv_unpack<<<(int)std::min<int64_t>(tiles, 8192), WG, 0, st>>>(P.bnd, lb, ub, (int32_t)n, Bp, V,
                                                                       L.wmask.as<uint8_t>(),
                                                                       P.base ? P.dmask : nullptr);
        HIPTRY(hipGetLastError());
        HIPTRY(hipStreamSynchronize(st));
    }
    return 0;
}

// A batch in pieces of at most 64 * LV_MAX_GROUPS vectors.
static int lv_propagate(bp_instance *h, int32_t B, double *lb, double *ub, const int32_t *idx,
                        const int64_t *ptr_dev, const std::vector<int64_t> &ptr, bool cold,
                        bp_result *res, hipStream_t st) {
    const int32_t maxv = 64 * LV_MAX_GROUPS;
    const int64_t n = h->n;
    for (int32_t v0 = 0; v0 < B; v0 += maxv) {
        const int32_t Bp = std::min(maxv, B - v0);
        const int64_t e0 = cold ? 0 : ptr[v0];
        const int64_t ec = cold ? 0 : ptr[v0 + Bp] - ptr[v0];
        if (int rc = lv_piece(h, Bp, lb + (size_t)v0 * n, ub + (size_t)v0 * n, idx,
                              cold ? nullptr : ptr_dev + v0, e0, ec, cold, res + v0, st))
            return rc;
    }
    return 0;
}
