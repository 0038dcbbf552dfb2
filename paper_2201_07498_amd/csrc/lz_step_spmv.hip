// The Lanczos-step SpMV and the standalone SpMV on gfx950 (Algorithm 1, the
// SpMV line): the kernels around the tile core of lz_spmv.h and their
// launchers.
#include <algorithm>
#include <cmath>

#include "lz_ooc.h"
#include "lz_spmv.h"

namespace lz {

// ------------------------------------------------------------------- SpMV
// Lanczos step SpMV (Algorithm 1, SpMV and alpha lines, and the beta term of
// the three-term update): y = scale_j * (A V[:,j]); w = y - beta_j v_{j-1};
// alpha_j = v_j . y in the one-pass modes.  In a restart iteration it draws
// the restart vector into w instead.
// Cached variant (mixed modes, large relabelled matrices): a workgroup of XW
// wavefronts first copies the head of x (the first XC_BYTES) into LDS.  After
// the hub-first relabelling the most frequently gathered entries sit there
// (on R-MAT scale 23 the first 16K columns take a third of all gathers), so
// those gathers skip L1 and L2.
constexpr int XW = 16;                 // wavefronts per workgroup of the cached variant
constexpr int XC_BYTES = 64 * 1024;

// Arithmetic of the epilogue (scale, beta term, alpha partials): double, or
// float in the all-FP32 mode.
template <bool F> struct Epi { using T = double; };
template <> struct Epi<true> { using T = float; };

// The solve's matrix is the caller's CSR (rp_a, col_a, val_a) or its
// relabelled copy (rp_b, ...), as the setup kernels decided.  Both come in as
// kernel arguments, so the compiler knows them to be global memory and emits
// global loads (pointers read from the state would give FLAT loads, which also
// count against the LDS counter).
// One launch covers tiles [tb, te).  A host-resident matrix takes one launch
// per slab (slab = 0 .. nslab-1, all with the same grid): col_a/val_a then
// point so that entry e of the matrix is col_a[e] for the slab's entries,
// launch `slab` writes its alpha partials after those of the earlier slabs,
// and the last launch reduces all of them.  A device-resident matrix is one
// slab of all tiles.  With SWEEP the relabelled matrix is walked in its
// sweep blocks (sw) instead of tiles.
template <int P, int NW, bool XCACHE, bool F = false, bool OFF32 = false, bool SWEEP = false>
__global__ __launch_bounds__(NW * 64) void k_spmv_step(State* st, const typename Tr<P>::V* __restrict__ Vb,
                                                       typename Tr<P>::W* __restrict__ w, int64_t n, int64_t nnz,
                                                       int64_t ld, int64_t n_tiles, const int32_t* __restrict__ ob,
                                                       uint32_t* tk, double* head, double* tail, double* part,
                                                       const int64_t* rp_a, const int32_t* col_a, const void* val_a,
                                                       const int64_t* rp_b, const int32_t* col_b, const void* val_b,
                                                       int64_t tb, int64_t te, int slab, int nslab,
                                                       int gate, SweepArgs sw) {
    using VT = typename Tr<P>::V;
    using AT = typename Tr<P>::A;
    using WT = typename Tr<P>::W;
    using E = typename Epi<F>::T;
    constexpr int H = XCACHE ? XC_BYTES / (int)sizeof(VT) : 1;
    __shared__ E shd[NW];
    __shared__ int s_last;
    __shared__ VT xs[H];
    if (st->status != 0) return;
    // Gated launch (the row order is decided on the device and the host does
    // not wait for it): gate 1 runs only on the relabelled matrix, gate 0 only
    // on the caller's, -1 always.
    if (gate >= 0 && (st->reordered != 0) != (gate == 1)) return;
    const int j = st->j;
    if (j >= st->m) return;
    if (st->mode == MODE_RESTART) {
        // Restart: a fresh random vector; the Gram-Schmidt kernels that follow
        // orthogonalise it against the basis.
        if (slab != 0) return;
        const uint64_t rs = st->seed + ((uint64_t)st->restarts << 32);
        const int32_t* perm = st->perm;
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += (int64_t)gridDim.x * blockDim.x)
            w[r] = (WT)(r < n ? u01(rs, (uint64_t)(perm ? perm[r] : r)) : 0.0);
        return;
    }
    const bool rl = st->reordered != 0;
    const int64_t* rp = rl ? rp_b : rp_a;
    const int32_t* col = rl ? col_b : col_a;
    const VT* val = (const VT*)(rl ? val_b : val_a);
    const VT* x = Vb + (int64_t)j * ld;
    const VT* xp = j > 0 ? Vb + (int64_t)(j - 1) * ld : nullptr;
    const E sj = (E)st->scale[j];
    const E bsc = j > 0 ? (E)st->beta[j] * (E)st->scale[j - 1] : E(0);
    E apart = E(0);
    // alpha = sum_r (sj x_r)(sj acc_r) is linear in every row sum, so a split
    // row adds one term per piece and the w update waits for the whole sum.
    // In the two-pass modes alpha comes from the first Gram-Schmidt pass
    // (alpha_j = c_j + beta_j v_j . v_{j-1}); only the other modes reduce it here.
    const bool need_alpha = st->reorth < 2;
    auto pre = [&](int64_t r) { return xp ? to_d(xp[r]) : 0.0; };
    auto row = [&](int64_t r, double acc, double xpr) {
        const E y = sj * (E)acc;
        if (need_alpha) apart += sj * (E)to_d(x[r]) * y;
        w[r] = (WT)(y - bsc * (E)xpr);
    };
    auto piece = [&](int64_t r, double acc) {
        if (need_alpha) apart += sj * (E)to_d(x[r]) * (sj * (E)acc);
    };
    auto fin = [&](int64_t r, double acc) { w[r] = (WT)(sj * (E)acc - (xp ? bsc * (E)to_d(xp[r]) : E(0))); };
    int hn = 0;
    if constexpr (XCACHE) {
        hn = (int)min<int64_t>(H, n);
        for (int i = threadIdx.x; i < hn; i += NW * 64) xs[i] = x[i];
        __syncthreads();
    }
    const int packing = rl ? st->packed : PACK_NONE;
    if constexpr (SWEEP) {
        if (packing != PACK_SWEEP) return;
        spmv_sweep<VT, NW, SweepShape<P>::ROWS>(sw, rp, x, n, tk, head, tail, pre, row, piece, fin);
    } else if (packing == PACK_GROUP) {
        spmv_groups<VT, AT, NW, XCACHE, OFF32>(rp, col, val, x, xs, hn, n, nnz, n_tiles, ob, tk, head, tail, pre,
                                               row, piece, fin);
    } else {
        spmv_tiles<VT, AT, NW, XCACHE, OFF32>(rp, col, val, x, xs, hn, n, nnz, n_tiles, tb, te,
                                              packing == PACK_TILE ? PACK_SLOTBITS : 0, ob, tk, head, tail, pre,
                                              row, piece, fin);
    }
    if (!need_alpha) return;
    apart = block_sum(apart, shd, NW);
    if (threadIdx.x == 0) st_dev(&part[(int64_t)slab * gridDim.x + blockIdx.x], (double)apart);
    if (slab != nslab - 1) return;
    __shared__ double shs[NW];
    if (last_block(&st->ticket[TK_SPMV], gridDim.x, &s_last)) {
        const double alpha = (double)(E)ordered_sum_dev(part, nslab * (int)gridDim.x, shs);
        if (threadIdx.x == 0) {
            st->alpha[j] = alpha;
            if (st->reorth == 0) {          // three-term recurrence only
                st->c2[j] = alpha;
                st->second = 1;
            }
        }
    }
}

// Plain y = A x (component entry point), same tiles and kernel core.
template <int P>
__global__ __launch_bounds__(BLOCK) void k_spmv_plain(State* st, const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const typename Tr<P>::V* __restrict__ val,
                                                      const typename Tr<P>::V* __restrict__ x,
                                                      typename Tr<P>::W* __restrict__ y, int64_t n, int64_t nnz,
                                                      int64_t n_tiles, const int32_t* __restrict__ ob, uint32_t* tk,
                                                      double* head, double* tail) {
    using VT = typename Tr<P>::V;
    using AT = typename Tr<P>::A;
    using WT = typename Tr<P>::W;
    if (st->status != 0) return;
    spmv_tiles<VT, AT, WAVES, false, false>(
        rp, col, val, x, nullptr, 0, n, nnz, n_tiles, 0, n_tiles, 0, ob, tk, head, tail,
        [](int64_t) { return 0.0; },
        [&](int64_t r, double acc, double) { y[r] = (WT)acc; }, [&](int64_t, double) {},
        [&](int64_t r, double acc) { y[r] = (WT)acc; });
}

// ---------------------------------------------------------------- launchers
template <int P, bool F = false>
static void spmv_step_p(const Plan& p, const Bufs& b, const Csr& a, hipStream_t s) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    // 32-bit byte offsets reach every entry of x.
    const bool off32 = (uint64_t)p.n * sizeof(VT) <= (uint64_t(1) << 32);
    if (p.sweep) {
        // Relabelled matrix: its sweep blocks; the caller's order takes the
        // tiles below (the x-head variant is not used with sweep blocks).
        using SS = SweepShape<P>;
        hipLaunchKernelGGL((k_spmv_step<P, SS::WAVES, false, F, false, true>), dim3(SS::GRID), dim3(SS::WAVES * 64),
                           0, s, b.st,
                           (const VT*)b.V, (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail,
                           b.part2, a.rowptr, a.col, a.val, b.rp2, b.col2, b.val2, (int64_t)0, p.n_tiles, 0, 1, 1,
                           SweepArgs{b.swob, b.swe, b.swcol, b.swrl, b.swval, p.sw_nb});
    }
    if constexpr (P != 0) {
        if (p.xcache && !p.sweep) {
            // One workgroup of XW wavefronts per CU (its LDS holds the x head).
            const int64_t g = std::min<int64_t>(256, (p.n_tiles + XW - 1) / XW);
            const int gx = (int)((g + 7) / 8 * 8);
            hipLaunchKernelGGL((k_spmv_step<P, XW, true, F>), dim3(gx), dim3(XW * 64), 0, s, b.st, (const VT*)b.V,
                               (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail, b.part2, a.rowptr,
                               a.col, a.val, b.rp2, b.col2, b.val2, (int64_t)0, p.n_tiles, 0, 1,
                               p.xcache == XC_GATED ? 1 : -1, SweepArgs{});
            if (p.xcache == XC_ON) return;
        }
    }
    {
        const int gate = (p.xcache == XC_GATED || p.sweep) ? 0 : -1;
        // FP32/BF16 storage: one resident set of workgroups (5 wavefronts per
        // SIMD, 256 CUs), each walking its share, so no late workgroups form
        // a tail (R-MAT 20 FP32: 80.1 -> 76.7 us).  FP64 does better the
        // other way, with one workgroup per four tiles up to 4096 (R-MAT 20:
        // 1024 -> 110.0 us, 2048 -> 106.8 us, 4096 -> 102.7 us).
        const int64_t g64 = std::min<int64_t>(4096, (p.n_tiles + 3) / 4);
        const int g = P == 0 ? (int)((g64 + 7) / 8 * 8) : std::min(p.g_tile, 5 * 256);
        if (off32)
            hipLaunchKernelGGL((k_spmv_step<P, WAVES, false, F, true>), dim3(g), dim3(BLOCK), 0, s, b.st,
                               (const VT*)b.V, (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail,
                               b.part2, a.rowptr, a.col, a.val, b.rp2, b.col2, b.val2, (int64_t)0, p.n_tiles, 0, 1,
                               gate, SweepArgs{});
        else
            hipLaunchKernelGGL((k_spmv_step<P, WAVES, false, F, false>), dim3(g), dim3(BLOCK), 0, s, b.st,
                               (const VT*)b.V, (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail,
                               b.part2, a.rowptr, a.col, a.val, b.rp2, b.col2, b.val2, (int64_t)0, p.n_tiles, 0, 1,
                               gate, SweepArgs{});
    }
}

// Host-resident matrix: one launch per slab, each on the slab's entries.
template <int P, bool F = false>
static hipError_t spmv_step_ooc(const Plan& p, const Bufs& b, const Csr& a, hipStream_t s) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    const bool off32 = (uint64_t)p.n * sizeof(VT) <= (uint64_t(1) << 32);
    return ooc_pass(*p.ooc, b.st, s, [&](const int32_t* col, const void* val, int64_t tb, int64_t te, int k, int ns) {
        if (off32)
            hipLaunchKernelGGL((k_spmv_step<P, WAVES, false, F, true>), dim3(p.g_slab), dim3(BLOCK), 0, s, b.st,
                               (const VT*)b.V, (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail,
                               b.part2, a.rowptr, col, val, nullptr, nullptr, nullptr, tb, te, k, ns, -1,
                               SweepArgs{});
        else
            hipLaunchKernelGGL((k_spmv_step<P, WAVES, false, F, false>), dim3(p.g_slab), dim3(BLOCK), 0, s, b.st,
                               (const VT*)b.V, (WT*)b.w, a.n, a.nnz, p.ld, p.n_tiles, b.ob, b.tk, b.head, b.tail,
                               b.part2, a.rowptr, col, val, nullptr, nullptr, nullptr, tb, te, k, ns, -1,
                               SweepArgs{});
    });
}

hipError_t launch_spmv_step(const Plan& p, const Bufs& b, const Csr& a, hipStream_t s) {
    if (p.ooc) {
        switch (p.prec) {
            case 0: return spmv_step_ooc<0>(p, b, a, s);
            case 1: return p.fff ? spmv_step_ooc<1, true>(p, b, a, s) : spmv_step_ooc<1>(p, b, a, s);
            default: return spmv_step_ooc<2>(p, b, a, s);
        }
    }
    switch (p.prec) {
        case 0: spmv_step_p<0>(p, b, a, s); break;
        case 1:
            if (p.fff)
                spmv_step_p<1, true>(p, b, a, s);
            else
                spmv_step_p<1>(p, b, a, s);
            break;
        default: spmv_step_p<2>(p, b, a, s); break;
    }
    return hipSuccess;
}

template <int P>
static void spmv_plain_p(const Plan& p, const Bufs& b, const Csr& a, const void* x, void* y, hipStream_t s) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    hipLaunchKernelGGL((k_spmv_plain<P>), dim3(p.g_tile), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                       (const VT*)a.val, (const VT*)x, (WT*)y, a.n, a.nnz, p.n_tiles, b.ob, b.tk, b.head, b.tail);
}

hipError_t launch_spmv_plain(const Plan& p, const Bufs& b, const Csr& a, const void* x, void* y, hipStream_t s) {
    switch (p.prec) {
        case 0: spmv_plain_p<0>(p, b, a, x, y, s); break;
        case 1: spmv_plain_p<1>(p, b, a, x, y, s); break;
        case 2: spmv_plain_p<2>(p, b, a, x, y, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lz
