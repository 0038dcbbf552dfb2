// CSR SpMV core over the row-partition work items (Algorithm 1, the SpMV
// line), shared by the Lanczos step, the standalone SpMV and the residual
// check.
//
// Work items are built once per matrix and are sized for one wavefront: a
// row block is a run of consecutive short rows with at most 2*NB non-zeros
// and RMAX = 64 rows; a long row (more than NB non-zeros) is cut into chunks
// of CH non-zeros.
//   Row block: every lane loads its col/val pairs first and then gathers x,
//     so all of a wavefront's loads are in flight together; the products are
//     staged in the wavefront's LDS slice and each row is summed by a
//     power-of-two group of lanes.
//   Long-row chunk: the wavefront sums CH products; chunk sums are published
//     device-coherently and the last chunk of the row to finish adds them in
//     chunk order.
// epi(r, acc, is_long, lid) receives every row sum exactly once: for a row
// block from its group leader lane, for a long row from lane 0 of the
// finalising wavefront.
#pragma once

#include "lz_device.h"

namespace lz {

constexpr int WAVES = BLOCK / 64;
constexpr int PPT = 2 * NB / 64;      // row-block products per lane

// Orders this wavefront's LDS writes before its later LDS reads (LDS
// operations of one wavefront complete in order; this stops the compiler
// from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// True in exactly one wavefront: the last of `count` to arrive.  Lane 0
// publishes the wavefront's partial (st_dev) before calling.
__device__ __forceinline__ bool last_wave(uint32_t* ticket, uint32_t count) {
    uint32_t t = 0;
    if ((threadIdx.x & 63) == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    t = __shfl(t, 0, 64);
    const bool last = t == count - 1u;
    if (last && (threadIdx.x & 63) == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return last;
}

// Each wavefront walks work items wid, wid + nwaves, ... independently (no
// workgroup barrier per item, so many items are in flight per CU).
template <class VT, class XT, class AT, class Epi>
__device__ __forceinline__ void spmv_items(State* st, const int64_t* __restrict__ rp,
                                           const int32_t* __restrict__ col, const VT* __restrict__ val,
                                           const XT* __restrict__ x, int nitems, const int2* __restrict__ items,
                                           const int32_t* __restrict__ lrow, const int32_t* __restrict__ lfirst,
                                           const int32_t* __restrict__ lnch, uint32_t* ltk, double* lpart,
                                           int wid, int nwaves, Epi&& epi) {
    __shared__ AT prod[WAVES][2 * NB];
    const int lane = threadIdx.x & 63;
    AT* pw = prod[threadIdx.x >> 6];
    for (int it = wid; it < nitems; it += nwaves) {
        const int2 item = items[it];
        if (item.x >= 0) {
            const int64_t rs = item.x, re = item.y;
            const int64_t ps = rp[rs];
            const int64_t cnt64 = rp[re] - ps;
            const int nr = (int)(re - rs);
            if (cnt64 < 0 || cnt64 > 2 * NB || nr > 64) {   // cannot happen for a validated partition
                if (lane == 0) st->status = -4;
                continue;
            }
            const int cnt = (int)cnt64;
            int tpr = 1;
            while (tpr < 64 && tpr * 2 * nr <= 64) tpr <<= 1;
            const int row = lane / tpr, sub = lane & (tpr - 1);
            int b0 = 0, e0 = 0;
            if (row < nr) {
                b0 = (int)(rp[rs + row] - ps);
                e0 = (int)(rp[rs + row + 1] - ps);
            }
            int ci[PPT];
            VT vv[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int t = lane + q * 64;
                if (t < cnt) {
                    ci[q] = col[ps + t];
                    vv[q] = val[ps + t];
                }
            }
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int t = lane + q * 64;
                if (t < cnt) pw[t] = to_a(vv[q], AT(0)) * to_a(x[ci[q]], AT(0));
            }
            wave_sync();
            AT s = AT(0);
            for (int k = b0 + sub; k < e0; k += tpr) s += pw[k];
            for (int o = tpr >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (row < nr && sub == 0) epi(rs + row, (double)s, false, 0);
            wave_sync();
        } else {
            const int lid = -1 - item.x;
            const int64_t r = lrow[lid];
            const int64_t p0 = rp[r] + (int64_t)item.y * CH;
            const int64_t p1 = min(p0 + (int64_t)CH, rp[r + 1]);
            const int cnt = (int)(p1 - p0);
            AT s = AT(0);
            for (int base = 0; base < cnt; base += PPT * 64) {
                int ci[PPT];
                VT vv[PPT];
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const int t = base + lane + q * 64;
                    if (t < cnt) {
                        ci[q] = col[p0 + t];
                        vv[q] = val[p0 + t];
                    }
                }
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const int t = base + lane + q * 64;
                    if (t < cnt) s += to_a(vv[q], AT(0)) * to_a(x[ci[q]], AT(0));
                }
            }
            s = wave_sum(s);
            if (lane == 0) st_dev(&lpart[it], (double)s);
            if (last_wave(&ltk[lid], (uint32_t)lnch[lid]) && lane == 0) {
                const int f = lfirst[lid], nc = lnch[lid];
                double tot = 0.0;
                for (int q = 0; q < nc; ++q) tot += ld_dev(&lpart[f + q]);
                epi(r, tot, true, lid);
            }
        }
    }
}

}  // namespace lz
