// bp_repair_run.h -- host side of the repair procedure (bp_repair and the
// repair step of bp_round); included by bp_engine.hip after bp_repair.h.
#pragma once

// The repair of the box lb/ub (device, in/out) inside the original box
// lb0/ub0 (device), inputs already checked.  res->status is BP_OK when
// repaired (lb/ub then hold the propagated box) and BP_INFEASIBLE when not
// (lb/ub untouched); res->reason says why (1 no improving candidate, 2
// shift limit, 3 attempt limit).
static int rp_run(bp_instance *h, double *lb, double *ub, const double *lb0, const double *ub0,
                  int32_t max_shifts, int32_t max_attempts, bp_repair_result *res, hipStream_t st) {
    memset(res, 0, sizeof(*res));
    res->status = BP_INFEASIBLE;
    const int64_t n = h->n, m = h->m;
    if (n == 0) {
        res->status = BP_OK;
        return 0;
    }
    ScWork W;
    int rc;
    if ((rc = sc_work_own(h, W))) return rc;
    if ((rc = h->rp_sums.grow((size_t)std::max<int64_t>(m, 1) * sizeof(RowSums), h->bytes))) return rc;
    if ((rc = h->rp_cand.grow((size_t)std::max<int64_t>(h->max_row_len, 1) * sizeof(RpCand), h->bytes)))
        return rc;
    if ((rc = h->rp_ctl.grow(sizeof(RpCtl), h->bytes))) return rc;
    if ((rc = h->rp_fixed.grow((size_t)n, h->bytes))) return rc;
    if ((rc = h->rp_pl.grow((size_t)n * 8, h->bytes))) return rc;
    if ((rc = h->rp_pu.grow((size_t)n * 8, h->bytes))) return rc;
    RowSums *sums = h->rp_sums.as<RowSums>();
    RpCand *cand = h->rp_cand.as<RpCand>();
    RpCtl *ctl = h->rp_ctl.as<RpCtl>();
    uint8_t *fixed = h->rp_fixed.as<uint8_t>();
    double *pl = h->rp_pl.as<double>(), *pu = h->rp_pu.as<double>();
    const DInst I = dinst_of(h);
    const double *cval = h->col_val.as<double>();
    const double feastol = h->opt.feastol, inttol = h->opt.inttol;
    const int rgrid = grid_for(std::max<int64_t>(m, 1));
    k_rp_fixed<<<grid_for(n), 256, 0, st>>>(h->vtype.as<uint8_t>(), lb, ub, n, fixed);
    k_pack<<<grid_for(n), 256, 0, st>>>(lb, ub, W.bnd, n, 1);
    HIPTRY(hipGetLastError());
    for (;;) {
        if ((rc = sc_rows_run(h, W, sums, st))) return rc;
        int32_t shifts = 0;
        for (;;) {
            RpCtl hc;
            k_rp_reset<<<1, 64, 0, st>>>(ctl);
            k_rp_viol_max<<<rgrid, 256, 0, st>>>(I, sums, feastol, ctl);
            k_rp_viol_row<<<rgrid, 256, 0, st>>>(I, sums, feastol, ctl);
            HIPTRY(hipGetLastError());
            HIPTRY(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
            HIPTRY(hipStreamSynchronize(st));
            if (hc.ebits == 0ull) break;
            if (shifts >= max_shifts) {
                res->reason = 2;
                return 0;
            }
            const int64_t L = h->row_len[hc.row];
            k_rp_cand<<<grid_for(L), 256, 0, st>>>(I, cval, sums, W.bnd, fixed, lb0, ub0, ctl, feastol,
                                                    inttol, cand);
            k_rp_best<<<1, RP_BEST, 0, st>>>(cand, L, ctl);
            HIPTRY(hipGetLastError());
            HIPTRY(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
            HIPTRY(hipStreamSynchronize(st));
            if (!hc.valid || !(hc.score < 0.0)) {
                res->reason = 1;
                return 0;
            }
            k_rp_apply<<<1, 64, 0, st>>>(ctl, W.bnd);
            HIPTRY(hipGetLastError());
            shifts += 1;
            res->shifts += 1;
            if ((rc = sc_rows_run(h, W, sums, st))) return rc;
        }
        // propagation of F's values from the original box (cold)
        k_rp_fixbox<<<grid_for(n), 256, 0, st>>>(W.bnd, fixed, lb0, ub0, n, pl, pu);
        HIPTRY(hipGetLastError());
        bp_result pr;
        if ((rc = propagate_slots(h, 1, pl, pu, nullptr, nullptr, 0, true, &pr, st, true)) < 0) return rc;
        res->attempts += 1;
        res->nnz_propagated += pr.nnz_propagated;
        if (pr.status != BP_INFEASIBLE) {
            HIPTRY(hipMemcpyAsync(lb, pl, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
            HIPTRY(hipMemcpyAsync(ub, pu, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
            HIPTRY(hipStreamSynchronize(st));
            res->status = BP_OK;
            res->reason = 0;
            return 0;
        }
        if (res->attempts >= max_attempts) {
            res->reason = 3;
            return 0;
        }
        // the next attempt starts from the same propagation one round
        // before the round that found it infeasible
        k_rp_fixbox<<<grid_for(n), 256, 0, st>>>(W.bnd, fixed, lb0, ub0, n, pl, pu);
        HIPTRY(hipGetLastError());
        if (pr.rounds > 1) {
            const int32_t saved = h->opt.max_rounds;
            h->opt.max_rounds = pr.rounds - 1;
            bp_result p2;
            rc = propagate_slots(h, 1, pl, pu, nullptr, nullptr, 0, true, &p2, st, true);
            h->opt.max_rounds = saved;
            if (rc < 0) return rc;
            res->nnz_propagated += p2.nnz_propagated;
        }
        k_pack<<<grid_for(n), 256, 0, st>>>(pl, pu, W.bnd, n, 1);
        HIPTRY(hipGetLastError());
    }
}

// Input checks of a repair: no NaN, lb0 <= ub0, the box inside the
// original box.
static int rp_check(bp_instance *h, const double *lb, const double *ub, const double *lb0,
                    const double *ub0, hipStream_t st) {
    if (h->n == 0) return 0;
    if (int rc = h->rp_ctl.grow(sizeof(RpCtl), h->bytes)) return rc;
    RpCtl *ctl = h->rp_ctl.as<RpCtl>();
    k_rp_reset<<<1, 64, 0, st>>>(ctl);
    k_rp_check<<<grid_for(h->n), 256, 0, st>>>(lb, ub, lb0, ub0, h->n, &ctl->bad);
    HIPTRY(hipGetLastError());
    int32_t bad = 0;
    HIPTRY(hipMemcpyAsync(&bad, &ctl->bad, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (bad) return fail(BP_EINVAL, "bp_repair: NaN bound, lb0 > ub0, or the box outside the original box");
    return 0;
}

extern "C" int bp_repair(bp_instance *h, double *lb, double *ub, const double *lb0, const double *ub0,
                         int32_t max_shifts, int32_t max_attempts, bp_repair_result *res,
                         void *stream) {
    BP_RANGE("bp_repair");
    BP_TABLES_CHECK(h);
    g_err.clear();
    if (!h || !res || (h->n > 0 && (!lb || !ub || !lb0 || !ub0)))
        return fail(BP_EINVAL, "bp_repair: null argument");
    if (max_shifts < 0 || max_attempts < 1)
        return fail(BP_EINVAL, "bp_repair: max_shifts must be >= 0 and max_attempts >= 1");
    hipStream_t st = as_stream(stream);
    if (int rc = rp_check(h, lb, ub, lb0, ub0, st)) return rc;
    bp_repair_result r;
    if (int rc = rp_run(h, lb, ub, lb0, ub0, max_shifts, max_attempts, &r, st)) return rc;
    *res = r;
    return BP_OK;
}
