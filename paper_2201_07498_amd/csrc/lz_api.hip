// C ABI of the Top-K Lanczos solver: argument checks, workspace planning and
// the launch sequence of one solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/lanczos_topk.h"
#include "lz_internal.h"
#include "lz_ooc.h"
#include "lz_solve.h"

namespace lz {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int pow2_ge(int k) {
    int v = 1;
    while (v < k) v <<= 1;
    return v;
}

Plan make_plan(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t prec, bool relabel, int sweep) {
    Plan p;
    p.n = n;
    p.nnz = nnz;
    p.K = K;
    p.m = m;
    p.prec = prec;
    // Leading dimension: a multiple of LDPAD, made an odd multiple so that the
    // same row of successive basis columns does not fall on the same HBM
    // channel (a power-of-two column stride sends them all to one).
    p.ld = ceil_div(n, LDPAD) * LDPAD;
    if ((p.ld / LDPAD) % 2 == 0) p.ld += LDPAD;
    p.KB = (int32_t)std::max<int64_t>(8, ceil_div(K, 8) * 8);
    p.g_orth = (int32_t)std::min<int64_t>(OGRID, p.ld / OBLOCK);
    p.g_dense = (int32_t)std::min<int64_t>(DGRID, p.ld / BLOCK);
    p.n_tiles = ceil_div(nnz + n, TILE);
    // Tiled SpMV grid: a multiple of 8 workgroups (one share per XCD).
    p.g_tile = (int32_t)(ceil_div(std::min<int64_t>(SGRID, ceil_div(p.n_tiles, 4)), 8) * 8);
    const int kb2 = pow2_ge(K);
    const size_t vb = storage_bytes(prec), wb = work_bytes(prec);
    // Scan scratch: the degree-class histogram (64 classes per 4096-row chunk).
    const int64_t scan_n = std::max<int64_t>(n, 64 * ceil_div(n, 4096));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    p.off_state = take(sizeof(State));
    p.off_V = take((size_t)p.ld * (size_t)(m + 1) * vb);
    p.off_w = take((size_t)p.ld * wb);
    p.off_part = take((size_t)std::max(p.g_dense, 1024) * 256 * 8);
    p.off_part2 = take((size_t)std::max(std::max(p.g_tile, p.g_dense), 2048) * 64 * 8);
    p.off_scan = take((size_t)scan_n * 8);
    p.off_bsum = take((size_t)(ceil_div(scan_n, 2048) + 2) * 8);
    p.off_Y = take((size_t)n * (size_t)K * 8);
    p.off_Z = take((size_t)n * (size_t)K * 8);
    p.off_gram = take((size_t)(GRAM_PARTS + 1) * 64 * 64 * 8);
    p.off_ob = take((size_t)(p.n_tiles + 1) * 4);
    p.off_tk = take((size_t)p.n_tiles * 4);
    p.off_head = take((size_t)p.n_tiles * kb2 * 8);
    p.off_tail = take((size_t)p.n_tiles * kb2 * 8);
    p.off_rp2 = take((size_t)(n + 1) * 8);
    p.off_col2 = take(relabel ? (size_t)nnz * 4 : 0);
    p.off_val2 = take(relabel ? (size_t)nnz * vb : 0);
    p.off_perm = take(relabel ? (size_t)n * 4 : 0);
    p.off_iperm = take(relabel ? (size_t)n * 4 : 0);
    p.off_gm = take((size_t)NCMAX * NCMAX * 8);
    p.sweep = relabel && sweep_applies(n, nnz, prec, sweep);
    if (p.sweep) {
        p.sw_items = (int64_t)SW_W * sweep_rows(prec);
        p.sw_nb = ceil_div(nnz + SW_W * n, p.sw_items);
        // Sort on the line of x an entry gathers (128 bytes), up to the
        // highest column bit.
        int bits = 0;
        while (bits < 31 && (int64_t(1) << bits) < n) ++bits;
        const int line = vb == 8 ? 4 : (vb == 4 ? 5 : 6);
        p.sw_bit1 = bits;
        p.sw_bit0 = line < bits ? line : 0;
        p.sw_sort_bytes = sweep_sort_bytes(nnz, p.sw_nb);
        p.off_swob = take((size_t)(p.sw_nb + 1) * 4);
        p.off_swe = take((size_t)(p.sw_nb + 1) * 8);
        p.off_swcol = take((size_t)nnz * 4);
        p.off_swrl = take((size_t)nnz * 2);
        p.off_swval = take((size_t)nnz * vb);
        p.off_swsrc = take((size_t)nnz * 4);
        p.off_swvin = take((size_t)nnz * 4);
        p.off_swtmp = take(p.sw_sort_bytes);
        p.off_swq = take(8 * 4);
    }
    p.bytes = o;
    return p;
}

Bufs resolve(const Plan& p, void* base) {
    char* c = (char*)base;
    Bufs b;
    b.st = (State*)(c + p.off_state);
    b.V = c + p.off_V;
    b.w = c + p.off_w;
    b.part = (double*)(c + p.off_part);
    b.part2 = (double*)(c + p.off_part2);
    b.scan = (uint64_t*)(c + p.off_scan);
    b.bsum = (uint64_t*)(c + p.off_bsum);
    b.Y = (double*)(c + p.off_Y);
    b.Z = (double*)(c + p.off_Z);
    b.gram = (double*)(c + p.off_gram);
    b.ob = (int32_t*)(c + p.off_ob);
    b.tk = (uint32_t*)(c + p.off_tk);
    b.head = (double*)(c + p.off_head);
    b.tail = (double*)(c + p.off_tail);
    b.rp2 = (int64_t*)(c + p.off_rp2);
    b.col2 = (int32_t*)(c + p.off_col2);
    b.val2 = c + p.off_val2;
    b.perm = (int32_t*)(c + p.off_perm);
    b.iperm = (int32_t*)(c + p.off_iperm);
    b.gm = (double*)(c + p.off_gm);
    b.swob = p.sweep ? (int32_t*)(c + p.off_swob) : nullptr;
    b.swe = p.sweep ? (int64_t*)(c + p.off_swe) : nullptr;
    b.swcol = p.sweep ? (int32_t*)(c + p.off_swcol) : nullptr;
    b.swrl = p.sweep ? (uint16_t*)(c + p.off_swrl) : nullptr;
    b.swval = p.sweep ? c + p.off_swval : nullptr;
    b.swsrc = p.sweep ? (uint32_t*)(c + p.off_swsrc) : nullptr;
    b.swvin = p.sweep ? (uint32_t*)(c + p.off_swvin) : nullptr;
    b.swtmp = p.sweep ? c + p.off_swtmp : nullptr;
    b.swq = p.sweep ? (uint32_t*)(c + p.off_swq) : nullptr;
    return b;
}

}  // namespace lz

using namespace lz;

#define LZ_HIP(call)                              \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) { rc = LZ_ERR_HIP; goto done; } \
    } while (0)

static int check_common(const void* rowptr, const void* col, const void* val, int64_t n, int32_t K, int32_t m,
                        int32_t precision) {
    if (!rowptr || !col || !val) return LZ_ERR_INVALID_ARG;
    if (n < 1 || n >= (int64_t(1) << 31)) return LZ_ERR_INVALID_ARG;
    if (precision < LZ_FP64 || precision > LZ_BF16) return LZ_ERR_INVALID_ARG;
    if (K < 1 || m < K || m > LZ_MAX_STEPS || (int64_t)m > n) return LZ_ERR_INVALID_ARG;
    return LZ_OK;
}

static int check_options(const lz_options* opt, int32_t precision, lz_options* out) {
    lz_options_init(out);
    if (opt) *out = *opt;
    const lz_options& o = *out;
    if (o.reorth < LZ_REORTH_NONE || o.reorth > LZ_REORTH_SELECTIVE) return LZ_ERR_INVALID_ARG;
    if (o.reorder < LZ_REORDER_OFF || o.reorder > LZ_REORDER_AUTO) return LZ_ERR_INVALID_ARG;
    if (o.arith < LZ_ARITH_MIXED || o.arith > LZ_ARITH_FP32) return LZ_ERR_INVALID_ARG;
    if (o.arith == LZ_ARITH_FP32 && precision != LZ_FP32) return LZ_ERR_INVALID_ARG;
    if (o.sweep < LZ_SWEEP_AUTO || o.sweep > LZ_SWEEP_ON) return LZ_ERR_INVALID_ARG;
    return LZ_OK;
}

// The plan of a device-resident solve with these options (the sweep-block
// copy only where the matrix may be relabelled).
static Plan plan_for(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision, const lz_options& o) {
    Plan p = make_plan(n, nnz, K, m, precision, true, o.reorder == LZ_REORDER_OFF ? LZ_SWEEP_OFF : o.sweep);
    p.fff = o.arith == LZ_ARITH_FP32;
    return p;
}

namespace lz {

int check_async(const int64_t* rowptr, const int32_t* col, const void* val, int64_t n, int64_t nnz, int32_t K,
                int32_t m, int32_t precision, const double* out_vals, const double* out_vecs,
                const lz_options* opt, lz_options* o, Plan* p, int* budget) {
    int rc = check_common(rowptr, col, val, n, K, m, precision);
    if (rc != LZ_OK) return rc;
    if (!out_vals || !out_vecs || nnz < 0 || nnz >= (int64_t(1) << 40)) return LZ_ERR_INVALID_ARG;
    rc = check_options(opt, precision, o);
    if (rc != LZ_OK) return rc;
    if (o->profile) return LZ_ERR_INVALID_ARG;
    *budget = o->max_restarts < 0 ? m : o->max_restarts;
    if (*budget > LZ_MAX_RESTART_BUDGET) return LZ_ERR_INVALID_ARG;
    *p = plan_for(n, nnz, K, m, precision, *o);
    return LZ_OK;
}

// The launch sequence of one solve, shared by the device-resident and the
// host-resident entry points (arguments already checked).  With hc, the
// matrix entries stay in host memory and a.rowptr is a host array.
int run_solve(Plan p, Csr a, const lz_options& o, hipStream_t s, double* out_vals, double* out_vecs,
              lz_report* report, HostCsr* hc) {
    const hipStream_t user = s;
    const int64_t n = a.n;
    const int32_t K = p.K, m = p.m;
    int rc = LZ_OK;
    void* ws = o.workspace;
    bool owned = false;
    State* hst = nullptr;
    // Profiling: phase events (start, after the start vector, after the
    // last Lanczos iteration, before and after the finish) and a pair around
    // the SpMV of every PROFILE_STRIDE-th iteration (the SpMV does the same
    // work at every step; each event adds a few microseconds of queue time,
    // so the steps in between run unbracketed).
    constexpr int PROFILE_STRIDE = 8;
    hipEvent_t pev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> iev;       // two per sampled iteration when profiling
    int launched = m;
    auto iter_events = [&](int t) -> hipEvent_t* {
        if (!o.profile || t % PROFILE_STRIDE != 0) return nullptr;
        const int slot = t / PROFILE_STRIDE;
        while ((int)iev.size() < 2 * (slot + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            iev.push_back(e);
        }
        return &iev[2 * slot];
    };
    {
        if (!ws) {
            if (hipMallocAsync(&ws, p.bytes, s) != hipSuccess) return LZ_ERR_OUT_OF_MEMORY;
            owned = true;
        }
        const Bufs b = resolve(p, ws);
        // Pinned host copy of the state (one per host thread, kept for the
        // process): pageable copies are staged in many small blits.
        static thread_local State* pinned = nullptr;
        if (!pinned && hipHostMalloc((void**)&pinned, sizeof(State), hipHostMallocDefault) != hipSuccess) {
            pinned = nullptr;
            rc = LZ_ERR_OUT_OF_MEMORY;
            goto done;
        }
        hst = pinned;
        if (o.profile) {
            for (int i = 0; i < 5; ++i) LZ_HIP(hipEventCreate(&pev[i]));
            LZ_HIP(hipEventRecord(pev[0], s));
        }
        if (hc) {
            const hipError_t be = ooc_begin(hc->ooc, &s);
            if (be != hipSuccess) {
                rc = LZ_ERR_HIP;
                goto done;
            }
            // Row pointers to the device (the slot of the relabelled ones).
            LZ_HIP(hipMemcpyAsync(b.rp2, a.rowptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
            a.rowptr = b.rp2;
        }
        LZ_HIP(launch_setup(p, b, a, o.seed, o.reorth, hc ? LZ_REORDER_OFF : o.reorder, s));
        if (hc) {
            const hipError_t pe = ooc_prepare(p, b, hc->ooc, hc->slab_nnz, hc->resident_nnz, s);
            if (pe == hipErrorOutOfMemory) {
                rc = LZ_ERR_OUT_OF_MEMORY;
                goto done;
            }
            LZ_HIP(pe);
            p.ooc = &hc->ooc;
        }
        if (!hc && o.reorder != LZ_REORDER_OFF && !p.sweep && want_xcache(p, true)) {
            // The SpMV variant depends on the row order the device chose.
            LZ_HIP(hipMemcpyAsync(hst, b.st, offsetof(State, maxdeg), hipMemcpyDeviceToHost, s));
            LZ_HIP(hipStreamSynchronize(s));
            p.xcache = want_xcache(p, hst->reordered != 0);
        }
        LZ_HIP(launch_init(p, b, s));
        if (o.profile) LZ_HIP(hipEventRecord(pev[1], s));
        for (int t = 0; t < m; ++t) LZ_HIP(launch_iteration(p, b, a, t + 1, o.reorth, s, iter_events(t)));
        if (o.profile) LZ_HIP(hipEventRecord(pev[2], s));
        // Breakdowns consume iterations without advancing j: run more until
        // m steps are done (bounded; each round advances j).
        for (int round = 0; round < 2 * LZ_MAX_STEPS + 2; ++round) {
            LZ_HIP(hipMemcpyAsync(hst, b.st, STATE_HEAD_BYTES, hipMemcpyDeviceToHost, s));
            LZ_HIP(hipStreamSynchronize(s));
            if (hst->status != 0 || hst->j >= m) break;
            const int extra = m - hst->j;
            for (int t = 0; t < extra; ++t)
                LZ_HIP(launch_iteration(p, b, a, m, o.reorth, s, iter_events(launched + t)));
            launched += extra;
            if (o.profile) LZ_HIP(hipEventRecord(pev[2], s));
        }
        if (hst->status == 0 && hst->j < m) {
            rc = LZ_ERR_BREAKDOWN;
            goto done;
        }
        if (o.profile) LZ_HIP(hipEventRecord(pev[3], s));
        if (hst->status == 0) LZ_HIP(launch_finish(p, b, a, out_vals, out_vecs, o.report, s));
        if (o.profile) LZ_HIP(hipEventRecord(pev[4], s));
        LZ_HIP(hipMemcpyAsync(hst, b.st, STATE_REPORT_BYTES, hipMemcpyDeviceToHost, s));
        LZ_HIP(hipStreamSynchronize(s));
        rc = hst->status;
        if (report) {
            std::memset(report, 0, sizeof(*report));
            report->status = hst->status;
            report->m_eff = std::min(hst->j, m);
            report->restarts = hst->restarts;
            report->jacobi_sweeps = hst->sweeps;
            report->beta_last = hst->beta[m];
            for (int k = 0; k < K; ++k) {
                report->resid[k] = hst->resid[k];
                report->abs_resid[k] = hst->abs_resid[k];
            }
            for (int i = 0; i < m; ++i) {
                report->alpha[i] = hst->alpha[i];
                report->theta[i] = hst->theta[i];
            }
            for (int i = 0; i <= m; ++i) report->beta[i] = hst->beta[i];
            report->ortho_loss = hst->ortho_loss;
            report->ritz_ortho_loss = hst->ritz_ortho_loss;
            report->mean_angle_deg = hst->mean_angle_deg;
            report->reordered = hst->reordered;
            report->spmv_layout = (hst->reordered ? 1 + hst->packed : 0) | (p.xcache ? LZ_LAYOUT_XCACHE : 0);
            report->bytes_streamed = hc ? hc->ooc.streamed : 0;
            if (o.profile && launched > 0) {
                float ms = 0.f;
                double sp = 0.0;
                int ns = 0;
                for (size_t i = 0; i + 1 < iev.size(); i += 2)
                    if (hipEventElapsedTime(&ms, iev[i], iev[i + 1]) == hipSuccess) {
                        sp += ms;
                        ++ns;
                    }
                report->t_spmv_ms = ns ? sp / ns : 0.0;
                if (hipEventElapsedTime(&ms, pev[0], pev[1]) == hipSuccess) report->t_setup_ms = ms;
                if (hipEventElapsedTime(&ms, pev[1], pev[2]) == hipSuccess) report->t_lanczos_ms = ms;
                if (hipEventElapsedTime(&ms, pev[3], pev[4]) == hipSuccess) report->t_finish_ms = ms;
                // The rest of a step: reorthogonalisation and launch gaps.
                report->t_orth_ms = std::max(0.0, report->t_lanczos_ms / launched - report->t_spmv_ms);
            }
        }
    }
done:
    if (owned || hc) (void)hipStreamSynchronize(s);
    if (hc) {
        if (hc->ooc.ks && ooc_end(hc->ooc, user) != hipSuccess && rc == LZ_OK) rc = LZ_ERR_HIP;
        ooc_release(hc->ooc);
    }
    if (owned) {
        (void)hipFreeAsync(ws, s);
        (void)hipStreamSynchronize(s);
    }
    for (hipEvent_t e : iev) (void)hipEventDestroy(e);
    for (hipEvent_t e : pev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// The results of a solve as an lz_report in device memory (stream-ordered
// calls): status, step and restart counts, the Lanczos coefficients, Ritz
// values, residuals and orthogonality metrics, as the blocking calls fill it
// on the host; no timings.
__global__ __launch_bounds__(BLOCK) void k_report(const State* st, lz_report* r, int xcache_if_relabelled) {
    const int m = st->m, K = st->K, t = threadIdx.x;
    if (t == 0) {
        r->status = st->status;
        r->m_eff = min(st->j, m);
        r->restarts = st->restarts;
        r->jacobi_sweeps = st->sweeps;
        r->beta_last = st->beta[m];
        r->ortho_loss = st->ortho_loss;
        r->ritz_ortho_loss = st->ritz_ortho_loss;
        r->mean_angle_deg = st->mean_angle_deg;
        r->t_setup_ms = r->t_lanczos_ms = r->t_spmv_ms = r->t_orth_ms = r->t_finish_ms = 0.0;
        r->reordered = st->reordered;
        r->spmv_layout = st->reordered ? (1 + st->packed) | (xcache_if_relabelled ? LZ_LAYOUT_XCACHE : 0) : 0;
        r->bytes_streamed = 0;
    }
    for (int i = t; i < LZ_MAX_STEPS; i += blockDim.x) {
        r->resid[i] = i < K ? st->resid[i] : 0.0;
        r->abs_resid[i] = i < K ? st->abs_resid[i] : 0.0;
        r->alpha[i] = i < m ? st->alpha[i] : 0.0;
        r->theta[i] = i < m ? st->theta[i] : 0.0;
    }
    for (int i = t; i <= LZ_MAX_STEPS; i += blockDim.x) r->beta[i] = i <= m ? st->beta[i] : 0.0;
}

hipError_t launch_report(const Plan&, const Bufs& b, void* d_report, int xcache_if_relabelled, hipStream_t s) {
    hipLaunchKernelGGL(k_report, dim3(1), dim3(BLOCK), 0, s, b.st, (lz_report*)d_report, xcache_if_relabelled);
    return hipGetLastError();
}

// Stream-ordered solve: every step is enqueued on `s` and nothing waits for
// the device.  The number of iterations is fixed when they are enqueued: m,
// plus `budget` more that absorb breakdowns (each restart takes one
// iteration that does not advance the step); iterations past the m-th step
// return at once.  The row-order decision is made on the device, so both
// SpMV variants that could apply are launched and each returns unless it
// matches.  ws: the caller's workspace, or null to allocate one
// stream-ordered (hipMallocAsync / hipFreeAsync on s).
int run_solve_async(Plan p, Csr a, const lz_options& o, int budget, hipStream_t s, double* out_vals,
                    double* out_vecs, void* d_report, void* ws) {
    int rc = LZ_OK;
    bool owned = false;
    if (!ws) {
        if (hipMallocAsync(&ws, p.bytes, s) != hipSuccess) return LZ_ERR_OUT_OF_MEMORY;
        owned = true;
    }
    {
        const Bufs b = resolve(p, ws);
        p.strict_m = 1;
        p.xcache = (o.reorder != LZ_REORDER_OFF && !p.sweep && want_xcache(p, true)) ? XC_GATED : XC_OFF;
        LZ_HIP(launch_setup(p, b, a, o.seed, o.reorth, o.reorder, s));
        LZ_HIP(launch_init(p, b, s));
        for (int t = 0; t < p.m; ++t) LZ_HIP(launch_iteration(p, b, a, t + 1, o.reorth, s));
        for (int t = 0; t < budget; ++t) LZ_HIP(launch_iteration(p, b, a, p.m, o.reorth, s));
        LZ_HIP(launch_finish(p, b, a, out_vals, out_vecs, o.report, s));
        if (d_report) LZ_HIP(launch_report(p, b, d_report, p.xcache != XC_OFF, s));
    }
done:
    if (owned && hipFreeAsync(ws, s) != hipSuccess && rc == LZ_OK) rc = LZ_ERR_HIP;
    return rc;
}

}  // namespace lz

extern "C" {

void lz_options_init(lz_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->seed = 0;
    opt->reorth = LZ_REORTH_TWICE;
    opt->report = 1;
    opt->reorder = LZ_REORDER_AUTO;
    opt->max_restarts = -1;
    opt->sweep = LZ_SWEEP_AUTO;
}

const char* lz_status_string(int status) {
    switch (status) {
        case LZ_OK: return "ok";
        case LZ_ERR_INVALID_ARG: return "invalid argument";
        case LZ_ERR_OUT_OF_MEMORY: return "out of device memory";
        case LZ_ERR_HIP: return "HIP runtime error";
        case LZ_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case LZ_ERR_TOO_LARGE: return "request larger than the memory budget";
        case LZ_ERR_NOT_CONVERGED: return "Jacobi did not converge";
        case LZ_ERR_NONFINITE: return "non-finite value in the Lanczos recurrence";
        case LZ_ERR_BREAKDOWN: return "restart vector lies in the Krylov basis";
        case LZ_ERR_RESTART_BUDGET: return "more breakdowns than the stream-ordered call's restart budget";
        case LZ_PENDING: return "pending";
        default: return "unknown status";
    }
}

size_t lanczos_topk_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision) {
    if (n < 1 || nnz < 0 || K < 1 || m < K || m > LZ_MAX_STEPS || precision < 0 || precision > 2) return 0;
    return make_plan(n, nnz, K, m, precision).bytes;
}

size_t lanczos_topk_workspace_size_opt(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision,
                                       const lz_options* opt) {
    if (n < 1 || nnz < 0 || K < 1 || m < K || m > LZ_MAX_STEPS || precision < 0 || precision > 2) return 0;
    lz_options o;
    if (check_options(opt, precision, &o) != LZ_OK) return 0;
    return plan_for(n, nnz, K, m, precision, o).bytes;
}

int lanczos_topk_ex(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val, int64_t n, int64_t nnz,
                    int32_t K, int32_t m, int32_t precision, void* stream, double* out_vals, double* out_vecs,
                    const lz_options* opt, lz_report* report) {
    int rc = check_common(csr_rowptr, csr_col, csr_val, n, K, m, precision);
    if (rc != LZ_OK) return rc;
    if (!out_vals || !out_vecs || nnz < 0 || nnz >= (int64_t(1) << 40)) return LZ_ERR_INVALID_ARG;
    lz_options o;
    rc = check_options(opt, precision, &o);
    if (rc != LZ_OK) return rc;
    Plan p = plan_for(n, nnz, K, m, precision, o);
    if (o.workspace && o.workspace_bytes < p.bytes) return LZ_ERR_WORKSPACE_TOO_SMALL;
    return run_solve(p, Csr{csr_rowptr, csr_col, csr_val, n, nnz}, o, (hipStream_t)stream, out_vals, out_vecs,
                     report, nullptr);
}

int lanczos_topk_async(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val, int64_t n,
                       int64_t nnz, int32_t K, int32_t m, int32_t precision, void* stream, double* out_vals,
                       double* out_vecs, const lz_options* opt, lz_report* d_report) {
    lz_options o;
    Plan p;
    int budget = 0;
    const int rc = check_async(csr_rowptr, csr_col, csr_val, n, nnz, K, m, precision, out_vals, out_vecs, opt, &o,
                               &p, &budget);
    if (rc != LZ_OK) return rc;
    if (o.workspace && o.workspace_bytes < p.bytes) return LZ_ERR_WORKSPACE_TOO_SMALL;
    return run_solve_async(p, Csr{csr_rowptr, csr_col, csr_val, n, nnz}, o, budget, (hipStream_t)stream, out_vals,
                           out_vecs, d_report, o.workspace);
}

int lz_check_symmetric(const int64_t* rowptr, const int32_t* col, const void* val, int64_t n, int32_t precision,
                       double rtol, int64_t* bad_row) {
    if (!rowptr || n < 1 || precision < LZ_FP64 || precision > LZ_BF16 || !(rtol >= 0.0)) return LZ_ERR_INVALID_ARG;
    const int64_t nnz = rowptr[n];
    if (rowptr[0] != 0 || nnz < 0 || (nnz > 0 && (!col || !val))) return LZ_ERR_INVALID_ARG;
    for (int64_t r = 0; r < n; ++r)
        if (rowptr[r + 1] < rowptr[r]) return LZ_ERR_INVALID_ARG;
    auto value = [&](int64_t e) -> double {
        if (precision == LZ_FP64) return ((const double*)val)[e];
        if (precision == LZ_FP32) return ((const float*)val)[e];
        const uint32_t u = (uint32_t)((const uint16_t*)val)[e] << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    // Canonical form: each row's entries sorted by column, duplicates summed.
    std::vector<int64_t> crp(n + 1, 0);
    std::vector<int32_t> cc;
    std::vector<double> cv;
    cc.reserve((size_t)nnz);
    cv.reserve((size_t)nnz);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t r = 0; r < n; ++r) {
        row.clear();
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n) return LZ_ERR_INVALID_ARG;
            row.emplace_back(col[e], value(e));
        }
        std::stable_sort(row.begin(), row.end(),
                         [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                             return x.first < y.first;
                         });
        for (size_t i = 0; i < row.size();) {
            double sum = 0.0;
            size_t k = i;
            for (; k < row.size() && row[k].first == row[i].first; ++k) sum += row[k].second;
            cc.push_back(row[i].first);
            cv.push_back(sum);
            i = k;
        }
        crp[r + 1] = (int64_t)cc.size();
    }
    // Transpose by counting; rows of the transpose come out column-sorted.
    std::vector<int64_t> trp(n + 1, 0);
    for (int32_t c : cc) ++trp[c + 1];
    for (int64_t r = 0; r < n; ++r) trp[r + 1] += trp[r];
    std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
    std::vector<int32_t> tc(cc.size());
    std::vector<double> tv(cc.size());
    for (int64_t r = 0; r < n; ++r)
        for (int64_t e = crp[r]; e < crp[r + 1]; ++e) {
            const int64_t at = fill[cc[e]]++;
            tc[at] = (int32_t)r;
            tv[at] = cv[e];
        }
    for (int64_t r = 0; r < n; ++r) {
        bool ok = crp[r + 1] - crp[r] == trp[r + 1] - trp[r];
        for (int64_t i = 0; ok && i < crp[r + 1] - crp[r]; ++i) {
            const int64_t a = crp[r] + i, b = trp[r] + i;
            ok = cc[a] == tc[b] && std::fabs(cv[a] - tv[b]) <= rtol * std::max(std::fabs(cv[a]), std::fabs(tv[b]));
        }
        if (!ok) {
            if (bad_row) *bad_row = r;
            return 0;
        }
    }
    return 1;
}

size_t lanczos_topk_host_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision) {
    if (n < 1 || nnz < 0 || K < 1 || m < K || m > LZ_MAX_STEPS || precision < 0 || precision > 2) return 0;
    return make_plan(n, nnz, K, m, precision, false).bytes;
}

int lanczos_topk_host(const int64_t* host_rowptr, const int32_t* host_col, const void* host_val, int64_t n,
                      int32_t K, int32_t m, int32_t precision, int64_t slab_nnz, int64_t resident_nnz, void* stream,
                      double* out_vals, double* out_vecs, const lz_options* opt, lz_report* report) {
    int rc = check_common(host_rowptr, host_col, host_val, n, K, m, precision);
    if (rc != LZ_OK) return rc;
    if (!out_vals || !out_vecs || resident_nnz < 0) return LZ_ERR_INVALID_ARG;
    const int64_t nnz = host_rowptr[n];
    if (host_rowptr[0] != 0 || nnz < 0 || nnz >= (int64_t(1) << 40)) return LZ_ERR_INVALID_ARG;
    if (slab_nnz == 0) slab_nnz = LZ_HOST_SLAB_NNZ_DEFAULT;
    // Every slab but the last holds more than slab_nnz - TILE entries.
    if (slab_nnz < 2 * TILE || nnz / (slab_nnz - TILE) + 2 > LZ_HOST_MAX_SLABS) return LZ_ERR_INVALID_ARG;
    lz_options o;
    rc = check_options(opt, precision, &o);
    if (rc != LZ_OK) return rc;
    if (o.reorder == LZ_REORDER_HUBS) return LZ_ERR_INVALID_ARG;
    Plan p = make_plan(n, nnz, K, m, precision, false);
    p.fff = o.arith == LZ_ARITH_FP32;
    if (o.workspace && o.workspace_bytes < p.bytes) return LZ_ERR_WORKSPACE_TOO_SMALL;
    // The entries are copied asynchronously while kernels run: they must be
    // pinned (page-locked) host memory.
    auto pinned_host = [](const void* ptr) {
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return at.type == hipMemoryTypeHost;
    };
    if (!pinned_host(host_col) || !pinned_host(host_val)) return LZ_ERR_INVALID_ARG;
    HostCsr hc;
    hc.slab_nnz = slab_nnz;
    hc.resident_nnz = resident_nnz;
    hc.ooc.hcol = host_col;
    hc.ooc.hval = (const char*)host_val;
    hc.ooc.vb = storage_bytes(precision);
    hc.ooc.n = n;
    return run_solve(p, Csr{host_rowptr, nullptr, nullptr, n, nnz}, o, (hipStream_t)stream, out_vals, out_vecs,
                     report, &hc);
}

int lanczos_topk(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val, int64_t n, int32_t K,
                 int32_t m, int32_t precision, void* stream, double* out_vals, double* out_vecs) {
    int rc = check_common(csr_rowptr, csr_col, csr_val, n, K, m, precision);
    if (rc != LZ_OK) return rc;
    int64_t nnz = -1;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&nnz, csr_rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LZ_ERR_HIP;
    return lanczos_topk_ex(csr_rowptr, csr_col, csr_val, n, nnz, K, m, precision, stream, out_vals, out_vecs,
                           nullptr, nullptr);
}

int lz_spmv(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val, int64_t n, int64_t nnz,
            int32_t precision, const void* x, void* y, void* stream) {
    if (!csr_rowptr || !csr_col || !csr_val || !x || !y) return LZ_ERR_INVALID_ARG;
    if (n < 1 || n >= (int64_t(1) << 31) || nnz < 0 || precision < 0 || precision > 2) return LZ_ERR_INVALID_ARG;
    const Plan p = make_plan(n, nnz, 1, 1, precision);
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    int rc = LZ_OK;
    State hst;
    if (hipMalloc(&ws, p.bytes) != hipSuccess) return LZ_ERR_OUT_OF_MEMORY;
    {
        const Bufs b = resolve(p, ws);
        const Csr a{csr_rowptr, csr_col, csr_val, n, nnz};
        LZ_HIP(launch_setup(p, b, a, 0, LZ_REORTH_TWICE, LZ_REORDER_OFF, s));
        LZ_HIP(launch_spmv_plain(p, b, a, x, y, s));
        LZ_HIP(hipMemcpyAsync(&hst, b.st, sizeof(State), hipMemcpyDeviceToHost, s));
        LZ_HIP(hipStreamSynchronize(s));
        rc = hst.status;
    }
done:
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
    return rc;
}

int lz_tridiag_eig(const double* alpha, const double* offdiag, int32_t m, double* theta, double* S, int32_t* sweeps) {
    if (!alpha || !theta || !S || m < 1 || m > LZ_MAX_STEPS || (m > 1 && !offdiag)) return LZ_ERR_INVALID_ARG;
    int rc = LZ_OK;
    char* d = nullptr;
    State* hst = new State;
    const size_t so = align_up(sizeof(State), 256);
    if (hipMalloc((void**)&d, so + 2 * 64 * 8) != hipSuccess) {
        delete hst;
        return LZ_ERR_OUT_OF_MEMORY;
    }
    {
        State* st = (State*)d;
        double* da = (double*)(d + so);
        double* dof = da + 64;
        LZ_HIP(hipMemcpy(da, alpha, m * 8, hipMemcpyHostToDevice));
        if (m > 1) LZ_HIP(hipMemcpy(dof, offdiag, (m - 1) * 8, hipMemcpyHostToDevice));
        LZ_HIP(launch_jacobi_only(da, dof, m, st, nullptr));
        LZ_HIP(hipMemcpy(hst, st, sizeof(State), hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i) theta[i] = hst->theta[i];
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) S[r * m + c] = hst->S[r * MMAX + c];
        if (sweeps) *sweeps = hst->sweeps;
        rc = hst->status;
    }
done:
    (void)hipFree(d);
    delete hst;
    return rc;
}

int lz_ortho_loss(const void* X, int64_t ldx, int64_t n, int32_t c, int32_t precision, void* stream,
                  double* out_loss) {
    if (!X || !out_loss || n < 1 || ldx < n || c < 1 || c > LZ_MAX_STEPS || precision < 0 || precision > 2)
        return LZ_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const size_t so = align_up(sizeof(State), 256);
    char* d = nullptr;
    int rc = LZ_OK;
    State* hst = new State;
    std::memset(hst, 0, sizeof(State));
    hst->j = c;
    hst->m = c;
    for (int k = 0; k < c; ++k) hst->scale[k] = 1.0;
    if (hipMalloc((void**)&d, so + (size_t)(GRAM_PARTS + 1) * 64 * 64 * 8) != hipSuccess) {
        delete hst;
        return LZ_ERR_OUT_OF_MEMORY;
    }
    {
        State* st = (State*)d;
        LZ_HIP(hipMemcpyAsync(st, hst, sizeof(State), hipMemcpyHostToDevice, s));
        LZ_HIP(launch_gram_only(precision, X, ldx, n, st, (double*)(d + so), s));
        LZ_HIP(hipMemcpyAsync(hst, st, sizeof(State), hipMemcpyDeviceToHost, s));
        LZ_HIP(hipStreamSynchronize(s));
        *out_loss = hst->ortho_loss;
    }
done:
    (void)hipStreamSynchronize(s);
    (void)hipFree(d);
    delete hst;
    return rc;
}

}  // extern "C"
