// Launch schedule of a context and the autotuner that picks it.
//
// None of the knobs changes a result: the block size only cuts the work queue differently, the
// launch widths only change how many workgroups share it, and the two DTW schedules (one lane per
// candidate, or one wave per candidate along anti-diagonals) compute the same recurrence.  The
// autotuner therefore checks that every schedule it times returns identical matches.
#include <chrono>
#include <cstring>
#include <vector>

#include "dtws_internal.h"

namespace {

constexpr int64_t kBlocks[] = {2048, 4096, 8192, 16384};
constexpr int32_t kDiagMaxes[] = {0, 2048, 16384, 65536};
constexpr int32_t kLbWidths[] = {4, 8, 16, 32};
constexpr int32_t kDtwWidths[] = {2, 4, 8};
constexpr int32_t kRounds[] = {4, 2, 1};
constexpr int32_t kEvicts[] = {4, 0, 2, 6};
constexpr int kKnobs = 11;
constexpr int kKnobValues[kKnobs] = {4, 4, 4, 3, 2, 2, 3, 2, 2, 2, 4};

bool valid_block(int64_t b) {
    if (b == 0) return true;
    for (int64_t x : kBlocks)
        if (b == x) return true;
    return false;
}

bool same(const std::vector<dtws_match> &a, const std::vector<dtws_match> &b) {
    for (size_t k = 0; k < a.size(); ++k)
        if (a[k].index != b[k].index || a[k].distance != b[k].distance || a[k].status != b[k].status) return false;
    return true;
}

}  // namespace

extern "C" {

DTWS_API int dtws_get_schedule(dtws_ctx *c, dtws_schedule *out) {
    if (!c || !out) return DTWS_EINVAL;
    out->block = c->block > 0 ? c->block : 4096;
    out->lb_blocks_per_cu = c->lb_blocks_per_cu > 0 ? c->lb_blocks_per_cu : 8;
    out->dtw_blocks_per_cu = c->dtw_blocks_per_cu > 0 ? c->dtw_blocks_per_cu : 4;
    out->diag_max = c->diag_max >= 0 ? c->diag_max : 16384;
    out->band_lanes = c->band_lanes;
    out->stats_prefix = c->stats_prefix;
    out->data_envelope = c->data_envelope;
    out->rounds = c->rounds;
    out->list_cap = c->list_cap;
    out->lb_tile = c->lb_tile;
    out->dtw_bound = c->dtw_bound;
    out->dtw_rows = c->dtw_rows;
    out->dtw_evict = c->dtw_evict;
    return DTWS_OK;
}

DTWS_API int dtws_set_schedule(dtws_ctx *c, const dtws_schedule *s) {
    if (!c || !s) return DTWS_EINVAL;
    if (!valid_block(s->block) || s->lb_blocks_per_cu < 0 || s->lb_blocks_per_cu > 64 || s->dtw_blocks_per_cu < 0 ||
        s->dtw_blocks_per_cu > 64 || s->diag_max < -1 || s->diag_max > (1 << 24) ||
        (s->band_lanes != 0 && s->band_lanes != 1 && s->band_lanes != 64) || (s->stats_prefix != 0 && s->stats_prefix != 1) ||
        (s->data_envelope != 0 && s->data_envelope != 1) || (s->rounds != 1 && s->rounds != 2 && s->rounds != 4) ||
        (s->list_cap != 0 && (s->list_cap < 64 || s->list_cap > (1 << 20))) || (s->lb_tile != 0 && s->lb_tile != 1) ||
        (s->dtw_bound != 0 && s->dtw_bound != 1) || (s->dtw_rows != 0 && s->dtw_rows != 1) ||
        s->dtw_evict < 0 || s->dtw_evict > 15)
        return DTWS_EINVAL;
    c->block = s->block;
    c->lb_blocks_per_cu = s->lb_blocks_per_cu;
    c->dtw_blocks_per_cu = s->dtw_blocks_per_cu;
    c->diag_max = s->diag_max;
    c->band_lanes = s->band_lanes;
    c->stats_prefix = s->stats_prefix;
    c->data_envelope = s->data_envelope;
    c->rounds = s->rounds;
    if (s->list_cap != c->list_cap && c->graph_exec) {
        // the capacity is baked into the captured graph's kernel arguments
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    c->list_cap = s->list_cap;
    c->lb_tile = s->lb_tile;
    c->dtw_bound = s->dtw_bound;
    c->dtw_rows = s->dtw_rows;
    c->dtw_evict = s->dtw_evict;
    return DTWS_OK;
}

DTWS_API int dtws_autotune_batch(dtws_ctx *c, const float *T, int64_t n, const float *Qp, const int64_t *qoff,
                                 const int32_t *mh, const int32_t *rh, int32_t nq, uint32_t flags, uint64_t seed,
                                 void *stream, int32_t reps, dtws_schedule *best_out, double *best_ms_out) {
    if (!c || !best_out || !best_ms_out || reps < 1 || reps > 100 || nq < 1 || nq > c->max_q) return DTWS_EINVAL;
    flags &= ~(uint32_t)DTWS_PROFILE;
    dtws_schedule start;
    memset(&start, 0, sizeof(start));
    dtws_get_schedule(c, &start);
    std::vector<dtws_match> ref(nq), got(nq);
    // one untimed call (it captures the graph), then `reps` timed calls
    auto run = [&](const dtws_schedule &sc, std::vector<dtws_match> &out, double &ms) -> int {
        int rc = dtws_set_schedule(c, &sc);
        if (rc != DTWS_OK) return rc;
        rc = dtws_search_batch(c, T, n, Qp, qoff, mh, rh, nq, flags, seed, stream, out.data());
        if (rc != DTWS_OK) return rc;
        const auto t0 = std::chrono::steady_clock::now();
        for (int k = 0; k < reps; ++k) {
            rc = dtws_search_batch(c, T, n, Qp, qoff, mh, rh, nq, flags, seed, stream, out.data());
            if (rc != DTWS_OK) return rc;
        }
        ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
        return DTWS_OK;
    };
    dtws_schedule best = start;
    double best_ms = 0.0;
    int rc = run(best, ref, best_ms);
    // coordinate descent: each knob in turn over its candidate values, keeping the fastest; then a
    // second pass over the knobs that interact most (the data envelope, the rounds and the tiled
    // cascade: with one of them changed, the best value of another often changes)
    auto sweep = [&](int knob) {
        const dtws_schedule base = best;
        for (int v = 0; v < kKnobValues[knob] && rc == DTWS_OK; ++v) {
            dtws_schedule t;
            memcpy(&t, &base, sizeof(t));
            switch (knob) {
            case 0: t.diag_max = kDiagMaxes[v]; break;
            case 1: t.block = kBlocks[v]; break;
            case 2: t.lb_blocks_per_cu = kLbWidths[v]; break;
            case 3: t.dtw_blocks_per_cu = kDtwWidths[v]; break;
            case 4: t.stats_prefix = v; break;
            case 5: t.data_envelope = 1 - v; break;
            case 6: t.rounds = kRounds[v]; break;
            case 7: t.lb_tile = 1 - v; break;
            case 8: t.dtw_bound = 1 - v; break;
            case 9: t.dtw_rows = 1 - v; break;
            default: t.dtw_evict = kEvicts[v]; break;
            }
            if (memcmp(&t, &base, sizeof(t)) == 0) continue;
            // the learned order keeps the block its model was trained with
            if (knob == 1 && (flags & DTWS_ORDER_MASK) == DTWS_ORDER_LEARNED && c->model_block > 0) continue;
            double ms = 0.0;
            rc = run(t, got, ms);
            if (rc != DTWS_OK) break;
            if (!same(ref, got)) {
                snprintf(c->lasterr, sizeof(c->lasterr), "autotune: schedules returned different matches");
                rc = DTWS_EHIP;
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    };
    for (int knob = 0; knob < kKnobs && rc == DTWS_OK; ++knob) sweep(knob);
    for (int knob : {5, 6, 7})
        if (rc == DTWS_OK) sweep(knob);
    if (rc != DTWS_OK) {
        dtws_set_schedule(c, &start);
        return rc;
    }
    dtws_set_schedule(c, &best);
    *best_out = best;
    *best_ms_out = best_ms;
    return DTWS_OK;
}

}  // extern "C"
