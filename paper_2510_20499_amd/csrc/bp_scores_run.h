// bp_scores_run.h -- host side of bp_scores and bp_probe_order (included by
// bp_engine.hip after the kernels of bp_scores.h).
#pragma once

// CSC values and the chunk table of the rows longer than 1024 nonzeros (the
// block and heavy bins), built once per instance.
static int sc_build(bp_instance *h, hipStream_t st) {
    if (h->sc_ready) return 0;
    const DInst I = dinst_of(h);
    if (int rc = h->sc_cval.alloc((size_t)std::max<int64_t>(h->nnz, 1) * 8, h->bytes)) return rc;
    if (h->n > 0) k_sc_cval<<<grid_for(h->n), 256, 0, st>>>(I, h->sc_cval.as<double>());
    HIPTRY(hipGetLastError());
    // long rows in bin order, from the cold-start row list
    std::vector<int32_t> cold((size_t)std::max<int32_t>(h->m, 1));
    if (h->m > 0)
        HIPTRY(hipMemcpyAsync(cold.data(), h->cold_rows.p, (size_t)h->m * 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
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
    if ((rc = h->sc_part.alloc(std::max<size_t>(chunks.size(), 1) * 2 * sizeof(Acc), h->bytes))) return rc;
    if (!rows.empty()) {
        HIPTRY(hipMemcpyAsync(h->sc_rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, st));
        HIPTRY(hipMemcpyAsync(h->sc_chunks.p, chunks.data(), chunks.size() * sizeof(int4),
                              hipMemcpyHostToDevice, st));
    }
    HIPTRY(hipMemcpyAsync(h->sc_first.p, first.data(), first.size() * 8, hipMemcpyHostToDevice, st));
    if ((rc = h->sc_act.alloc((size_t)std::max<int32_t>(h->m, 1) * sizeof(double2), h->bytes))) return rc;
    if ((rc = h->sc_bnd.alloc((size_t)std::max<int32_t>(h->n, 1) * 16, h->bytes))) return rc;
    HIPTRY(hipStreamSynchronize(st));
    h->sc_ready = true;
    return 0;
}

// Bounds in (NaN rejected), then the exact activity of every row.
static int sc_rows_pass(bp_instance *h, const double *lb, const double *ub, hipStream_t st) {
    const int64_t n = h->n;
    if (int rc = sc_build(h, st)) return rc;
    const DInst I = dinst_of(h);
    double2 *bnd = h->sc_bnd.as<double2>();
    if (n > 0) {
        k_pack<<<grid_for(n), 256, 0, st>>>(lb, ub, bnd, n, 1);
        if (int rc = h->idflag_d.grow(4, h->bytes)) return rc;
        int32_t zero = 0, bad = 0;
        HIPTRY(hipMemcpyAsync(h->idflag_d.p, &zero, 4, hipMemcpyHostToDevice, st));
        k_sc_nan<<<grid_for(n), 256, 0, st>>>(bnd, n, h->idflag_d.as<int32_t>());
        HIPTRY(hipGetLastError());
        HIPTRY(hipMemcpyAsync(&bad, h->idflag_d.p, 4, hipMemcpyDeviceToHost, st));
        HIPTRY(hipStreamSynchronize(st));
        if (bad) return fail(BP_EINVAL, "NaN bound");
    }
    double2 *act = h->sc_act.as<double2>();
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
        k_sc_rows<<<(int)std::min<int64_t>(units, 8192), WG, 0, st>>>(I, bnd, R, h->sc_part.as<Acc>(), act);
    if (h->sc_nlong > 0)
        k_sc_combine<<<(int)std::min<int64_t>((h->sc_nlong + 3) / 4, 4096), WG, 0, st>>>(
            I, bnd, h->sc_rows.as<int32_t>(), h->sc_first.as<int64_t>(), h->sc_nlong,
            h->sc_part.as<Acc>(), act);
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

extern "C" int bp_scores(bp_instance *h, const double *lb, const double *ub, bp_scores_out *out,
                         void *stream) {
    if (!h || !out) return fail(BP_EINVAL, "null argument");
    if (h->n > 0 && (!lb || !ub)) return fail(BP_EINVAL, "null bounds");
    hipStream_t st = as_stream(stream);
    if (int rc = sc_rows_pass(h, lb, ub, st)) return rc;
    if (h->n > 0)
        k_sc_vars<<<grid_for(h->n), 256, 0, st>>>(dinst_of(h), h->sc_bnd.as<double2>(),
                                                   h->sc_cval.as<double>(), h->sc_act.as<double2>(),
                                                   h->opt.feastol, out->nviol, out->maxviol,
                                                   out->minunit, out->slack_score);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    return BP_OK;
}

extern "C" int bp_probe_order(bp_instance *h, const double *lb, const double *ub,
                              const int32_t *vars, int32_t k, int32_t *order, void *stream) {
    if (!h || k < 0) return fail(BP_EINVAL, "bad argument");
    if (k > 0 && (!vars || !order)) return fail(BP_EINVAL, "null argument");
    if (h->n > 0 && (!lb || !ub)) return fail(BP_EINVAL, "null bounds");
    hipStream_t st = as_stream(stream);
    if (k > 0)
        if (int rc = check_ids(h, vars, k, st)) return rc;
    if (int rc = sc_rows_pass(h, lb, ub, st)) return rc;
    if (k == 0) return BP_OK;
    const int64_t n = h->n;
    // nviol | maxviol | minunit of every variable
    if (int rc = h->sc_tmp.grow((size_t)n * 20, h->bytes)) return rc;
    double *mv = h->sc_tmp.as<double>();
    double *mu = mv + n;
    int32_t *nv = (int32_t *)(mu + n);
    k_sc_vars<<<grid_for(n), 256, 0, st>>>(dinst_of(h), h->sc_bnd.as<double2>(), h->sc_cval.as<double>(),
                                           h->sc_act.as<double2>(), h->opt.feastol, nv, mv, mu,
                                           nullptr);
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
