// bp_round_run.h -- host loop of bp_round (included by bp_engine.hip after
// bp_round.h).
#pragma once

// Stable compaction of the flagged entries of [0, N) (values[i], or i) into
// out; the count lands in *total_d (device).
static int rd_compact(bp_instance *h, const uint8_t *flags, const int32_t *values, int64_t N,
                      int32_t *out, int64_t *total_d, hipStream_t st) {
    if (N == 0) {
        HIPTRY(hipMemsetAsync(total_d, 0, 8, st));
        return 0;
    }
    const int64_t nb = (N + CMP_BLOCK - 1) / CMP_BLOCK;
    if (int rc = h->rd_bcnt.grow((size_t)nb * 4, h->bytes)) return rc;
    int32_t *bcnt = h->rd_bcnt.as<int32_t>();
    const int grid = (int)std::min<int64_t>(nb, 4096);
    k_cmp_count<<<grid, WG, 0, st>>>(flags, N, bcnt);
    k_cmp_scan<<<1, WG, 0, st>>>(bcnt, nb, total_d);
    k_cmp_write<<<grid, WG, 0, st>>>(flags, values, N, bcnt, out);
    HIPTRY(hipGetLastError());
    return 0;
}

static int64_t pow2_at_least(int64_t k) {
    int64_t p = 1;
    while (p < k) p <<= 1;
    return p;
}

// Rounds per captured graph for the warm propagations of the rounding
// steps: a bulk settles in a few rounds, and the unused rounds of a graph
// still launch (as no-ops).
constexpr int32_t RD_ROUNDS_PER_LAUNCH = 4;

static int round_impl(bp_instance *h, double *lb, double *ub, const double *x, const double *draws,
                      const bp_cache *cache, bp_round_result *res, hipStream_t st);

extern "C" int bp_round(bp_instance *h, double *lb, double *ub, const double *x, const double *draws,
                        const bp_cache *cache, bp_round_result *res, void *stream) {
    BP_RANGE("bp_round");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !res || (h->n > 0 && (!lb || !ub || !x || !draws)))
        return fail(BP_EINVAL, "bp_round: null argument");
    const int32_t saved = h->opt.rounds_per_launch;
    h->opt.rounds_per_launch = std::min(saved, RD_ROUNDS_PER_LAUNCH);
    const int rc = round_impl(h, lb, ub, x, draws, cache, res, as_stream(stream));
    h->opt.rounds_per_launch = saved;
    return rc;
}

static int round_impl(bp_instance *h, double *lb, double *ub, const double *x, const double *draws,
                      const bp_cache *cache, bp_round_result *res, hipStream_t st) {
    if (cache && cache->k < 0) return fail(BP_EINVAL, "bp_round: negative cache size");
    if (cache && cache->k > 0 && (!cache->vars || !cache->status || !cache->off))
        return fail(BP_EINVAL, "bp_round: incomplete cache");
    const int64_t n = h->n;
    memset(res, 0, sizeof(*res));
    if (n == 0) return BP_OK;
    const int32_t k = cache ? cache->k : 0;
    int rc;
    // work buffers
    if ((rc = h->rd_order.grow((size_t)n * 4, h->bytes))) return rc;
    if ((rc = h->rd_order2.grow((size_t)n * 4, h->bytes))) return rc;
    if ((rc = h->rd_flags.grow((size_t)2 * n, h->bytes))) return rc;
    if ((rc = h->rd_small.grow(64, h->bytes))) return rc;
    if ((rc = h->rd_S.grow((size_t)n * 8, h->bytes))) return rc;
    if ((rc = h->rd_keys.grow((size_t)pow2_at_least(n) * sizeof(ScKey), h->bytes))) return rc;
    if ((rc = h->rd_val.grow((size_t)2 * n * 8, h->bytes))) return rc;
    if ((rc = h->rd_keep.grow((size_t)2 * n, h->bytes))) return rc;
    if ((rc = h->rd_mpos.grow((size_t)n * 4, h->bytes))) return rc;
    if ((rc = h->rd_mbox.grow((size_t)2 * n * 16, h->bytes))) return rc;
    if ((rc = h->rd_vk.grow((size_t)2 * n * 16, h->bytes))) return rc;
    if ((rc = h->rd_vl.grow((size_t)2 * n * 8, h->bytes))) return rc;
    if ((rc = h->rd_vu.grow((size_t)2 * n * 8, h->bytes))) return rc;
    if ((rc = h->rd_chg.grow((size_t)3 * n * 4, h->bytes))) return rc;
    if ((rc = h->rd_cpos.grow((size_t)n * 4, h->bytes))) return rc;
    if (h->opt.repair_calls > 0 && (rc = h->rd_start.grow((size_t)2 * n * 8, h->bytes))) return rc;
    int32_t *order = h->rd_order.as<int32_t>(), *order2 = h->rd_order2.as<int32_t>();
    uint8_t *flags = h->rd_flags.as<uint8_t>();
    int64_t *tot = h->rd_small.as<int64_t>();               // [0..1] counts
    int32_t *kept = (int32_t *)(h->rd_small.as<int64_t>() + 2);  // [2]
    int32_t *bad = kept + 2;
    int64_t *chg_ptr = h->rd_small.as<int64_t>() + 4;        // [3]
    double *S = h->rd_S.as<double>();
    ScKey *keys = h->rd_keys.as<ScKey>();
    double *val = h->rd_val.as<double>();
    uint8_t *keep = h->rd_keep.as<uint8_t>();
    int32_t *mpos = h->rd_mpos.as<int32_t>();
    longlong2 *mbox = h->rd_mbox.as<longlong2>(), *vk = h->rd_vk.as<longlong2>();
    double *vl = h->rd_vl.as<double>(), *vu = h->rd_vu.as<double>();
    int32_t *chg = h->rd_chg.as<int32_t>();
    const uint8_t *vtype = h->vtype.as<uint8_t>();
    // input checks
    HIPTRY(hipMemsetAsync(bad, 0, 4, st));
    k_rd_check<<<grid_for(std::max<int64_t>(2 * n, 2 * (int64_t)k + 1)), 256, 0, st>>>(
        x, draws, lb, ub, n, k ? cache->vars : nullptr, k, k ? cache->off : nullptr, bad);
    int32_t hbad = 0;
    HIPTRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (hbad) return fail(BP_EINVAL, "bp_round: NaN in x or the box, a draw outside [0, 1), or a "
                                     "malformed cache");
    if (k > 0) {
        // the cache's implied variables must be ids of this instance
        int64_t entries = 0;
        HIPTRY(hipMemcpyAsync(&entries, cache->off + 2 * (int64_t)k, 8, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (entries > 0 && (!cache->var || !cache->lb || !cache->ub))
            return fail(BP_EINVAL, "bp_round: incomplete cache");
        if (entries > 0)
            if ((rc = check_ids(h, cache->var, entries, st))) return rc;
    }
    // the box the rounding starts from: the repair's original box
    double *start_l = h->opt.repair_calls > 0 ? h->rd_start.as<double>() : nullptr;
    double *start_u = start_l ? start_l + n : nullptr;
    if (start_l) {
        HIPTRY(hipMemcpyAsync(start_l, lb, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
        HIPTRY(hipMemcpyAsync(start_u, ub, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
    }
    RdCache C;
    C.k = k;
    C.pos = h->rd_cpos.as<int32_t>();
    C.status = k ? cache->status : nullptr;
    C.off = k ? cache->off : nullptr;
    C.var = k ? cache->var : nullptr;
    C.lb = k ? cache->lb : nullptr;
    C.ub = k ? cache->ub : nullptr;
    k_fill_i32<<<grid_for(n), 256, 0, st>>>(h->rd_cpos.as<int32_t>(), -1, n);
    if (k > 0) k_rd_cache_pos<<<grid_for(k), 256, 0, st>>>(cache->vars, k, h->rd_cpos.as<int32_t>());
    k_fill_i32<<<grid_for(n), 256, 0, st>>>(mpos, -1, n);
    // unset variables in their initial order
    k_rd_flag_start<<<grid_for(n), 256, 0, st>>>(vtype, lb, ub, n, flags);
    if ((rc = rd_compact(h, flags, nullptr, n, order2, tot, st))) return rc;
    int64_t R = 0;
    HIPTRY(hipMemcpyAsync(&R, tot, 8, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (R > 0) {
        const int64_t kpad = pow2_at_least(R);
        k_rd_initial_keys<<<grid_for(kpad), 256, 0, st>>>(order2, R, kpad, x, lb, ub, keys);
        sc_sort(keys, kpad, st);
        k_rd_from_keys<<<grid_for(R), 256, 0, st>>>(keys, R, nullptr, order);
    }
    bool recovery = false, infeasible = false;
    const int64_t cap_iter = 2 * R + 16;
    std::vector<int64_t> hc(2);
    std::vector<int32_t> hk(2);
    bp_result pr[2];
    for (;;) {
        // the unfixed variables, in order
        if (R > 0) {
            k_rd_flag_unfixed<<<grid_for(R), 256, 0, st>>>(order, R, lb, ub, flags);
            if ((rc = rd_compact(h, flags, order, R, order2, tot, st))) return rc;
            HIPTRY(hipMemcpyAsync(&R, tot, 8, hipMemcpyDeviceToHost, st));
            HIPTRY(hipStreamSynchronize(st));
            std::swap(order, order2);
        }
        if (R == 0) break;
        if (res->iterations >= cap_iter) return fail(BP_EDEVICE, "bp_round: no progress");
        res->iterations += 1;
        int64_t bulk = (recovery || R <= 36) ? 1 : (int64_t)std::ceil(std::sqrt((double)R));
        if (bulk > 1) {
            // implied-slack re-sort (stable): S at the current box
            ScWork W;
            if ((rc = sc_work_own(h, W)) || (rc = sc_rows_pass(h, lb, ub, W, st))) return rc;
            k_sc_vars<<<grid_for(n), 256, 0, st>>>(dinst_of(h), W.bnd, h->col_val.as<double>(), W.act,
                                                   h->opt.feastol, nullptr, nullptr, nullptr, S);
            const int64_t kpad = pow2_at_least(R);
            k_rd_slack_keys<<<grid_for(kpad), 256, 0, st>>>(order, R, kpad, S, keys);
            sc_sort(keys, kpad, st);
            k_rd_from_keys<<<grid_for(R), 256, 0, st>>>(keys, R, order, order2);
            std::swap(order, order2);
        }
        if (bulk > R) bulk = R;
        // values, cache conflicts, warm starts
        HIPTRY(hipMemsetAsync(kept, 0, 8, st));
        k_rd_values<<<grid_for(bulk), 256, 0, st>>>(order, bulk, x, draws, lb, ub, C, val, keep, mpos,
                                                    mbox);
        if (k > 0)
            k_rd_member_boxes<<<grid_for(2 * bulk), 256, 0, st>>>(order, bulk, C, val, keep, mpos, mbox);
        k_rd_member_check<<<grid_for(bulk), 256, 0, st>>>(order, bulk, val, keep, mpos, mbox, kept);
        k_rd_warm_init<<<grid_for(n), 256, 0, st>>>(lb, ub, n, vk);
        if (k > 0)
            k_rd_warm_implied<<<grid_for(2 * bulk), 256, 0, st>>>(order, bulk, C, val, keep, n, vk);
        k_rd_warm_fix<<<grid_for(2 * bulk), 256, 0, st>>>(order, bulk, val, keep, n, vk);
        k_rd_warm_out<<<grid_for(2 * n), 256, 0, st>>>(vk, lb, ub, n, vl, vu, flags);
        // changed lists: vector 0 at chg, vector 1 at chg + 2n, then packed
        // behind vector 0's (the regions cannot overlap)
        if ((rc = rd_compact(h, flags, nullptr, n, chg, tot, st))) return rc;
        if ((rc = rd_compact(h, flags + n, nullptr, n, chg + 2 * n, tot + 1, st))) return rc;
        // counts and kept members in one read (rd_small bytes 0..23)
        int64_t small[3];
        HIPTRY(hipMemcpyAsync(small, tot, 24, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        hc[0] = small[0];
        hc[1] = small[1];
        memcpy(hk.data(), &small[2], 8);
        if (hc[1] > 0)
            HIPTRY(hipMemcpyAsync(chg + hc[0], chg + 2 * n, (size_t)hc[1] * 4, hipMemcpyDeviceToDevice, st));
        bool ok[2] = {false, false};
        if (hk[0] > 0 || hk[1] > 0) {
            const int64_t hptr[3] = {0, hc[0], hc[0] + hc[1]};
            HIPTRY(hipMemcpyAsync(chg_ptr, hptr, 24, hipMemcpyHostToDevice, st));
            // the changed ids come from the compaction: no range check
            if ((rc = propagate_slots(h, 2, vl, vu, chg, chg_ptr, hc[0] + hc[1], false, pr, st, true)) < 0)
                return rc;
            for (int q = 0; q < 2; ++q) {
                if (hk[q] == 0) continue;
                res->nnz_propagated += pr[q].nnz_propagated;
                ok[q] = pr[q].status != BP_INFEASIBLE;
            }
        }
        if (bulk > 1) res->bulks += 1;
        else res->singles += 1;
        if (ok[0] || ok[1]) {
            const int q = ok[0] ? 0 : 1;
            HIPTRY(hipMemcpyAsync(lb, vl + q * n, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
            HIPTRY(hipMemcpyAsync(ub, vu + q * n, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
            recovery = false;
        } else {
            if (!recovery && !infeasible) {
                recovery = true;
                res->recoveries += 1;
            } else {
                infeasible = true;
            }
            if (infeasible) {
                k_rd_fix_first<<<grid_for(bulk), 256, 0, st>>>(order, bulk, val, lb, ub);
                recovery = false;
            }
        }
        HIPTRY(hipGetLastError());
        // Algorithm 1: on a marked path every step ends with a repair until
        // one succeeds or the allowed repairs are spent
        if (infeasible && res->repairs < h->opt.repair_calls) {
            bp_repair_result rr;
            if ((rc = rp_run(h, lb, ub, start_l, start_u, h->opt.repair_shifts, h->opt.repair_attempts,
                             &rr, st)) < 0)
                return rc;
            res->repairs += 1;
            res->nnz_propagated += rr.nnz_propagated;
            if (rr.status == BP_OK) {
                res->repaired += 1;
                infeasible = false;
            }
        }
    }
    res->status = infeasible ? BP_INFEASIBLE : BP_OK;
    // integer variables fixed at the end
    k_rd_flag_fixed<<<grid_for(n), 256, 0, st>>>(vtype, lb, ub, n, flags);
    if ((rc = rd_compact(h, flags, nullptr, n, order2, tot, st))) return rc;
    int64_t fixed = 0;
    HIPTRY(hipMemcpyAsync(&fixed, tot, 8, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    res->fixed = (int32_t)fixed;
    return BP_OK;
}
