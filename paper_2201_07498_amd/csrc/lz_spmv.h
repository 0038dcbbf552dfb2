// CSR SpMV core over the row-partition work items (Algorithm 1, the SpMV
// line), shared by the Lanczos step, the standalone SpMV and the residual
// check.
//
// Work items are built once per matrix: a row block is a run of consecutive
// short rows with at most 2*NB non-zeros and RMAX rows; a long row (more than
// NB non-zeros) is cut into chunks of CH non-zeros.
//   Row block: every lane loads its col/val pairs first and then gathers x,
//     so all of a workgroup's loads are in flight together; the products are
//     staged in LDS and each row is summed by a power-of-two group of lanes.
//   Long-row chunk: the workgroup sums CH products; chunk sums are published
//     device-coherently and the last chunk of the row to finish adds them in
//     chunk order.
// epi(r, acc, is_long, lid) receives every row sum exactly once: for a row
// block from its group leader, for a long row from thread 0 of the
// finalising workgroup.
#pragma once

#include "lz_device.h"

namespace lz {

constexpr int PPT = 2 * NB / BLOCK;   // row-block products per thread

template <class VT, class XT, class AT, class Epi>
__device__ __forceinline__ void spmv_items(State* st, const int64_t* __restrict__ rp,
                                           const int32_t* __restrict__ col, const VT* __restrict__ val,
                                           const XT* __restrict__ x, int nitems, const int2* __restrict__ items,
                                           const int32_t* __restrict__ lrow, const int32_t* __restrict__ lfirst,
                                           const int32_t* __restrict__ lnch, uint32_t* ltk, double* lpart,
                                           int bid, int nblk, Epi&& epi) {
    __shared__ AT prod[2 * NB];
    __shared__ AT sha[BLOCK / 64];
    __shared__ int s_last;
    const int tid = threadIdx.x;
    for (int it = bid; it < nitems; it += nblk) {
        const int2 item = items[it];
        if (item.x >= 0) {
            const int64_t rs = item.x, re = item.y;
            const int64_t ps = rp[rs];
            const int64_t cnt64 = rp[re] - ps;
            if (cnt64 < 0 || cnt64 > 2 * NB) {          // cannot happen for a validated partition
                if (tid == 0) st->status = -4;
                continue;
            }
            const int cnt = (int)cnt64;
            const int nr = (int)(re - rs);
            int tpr = 1;
            while (tpr < 64 && tpr * 2 * nr <= BLOCK) tpr <<= 1;
            const int row = tid / tpr, lane = tid & (tpr - 1);
            int b0 = 0, e0 = 0;
            if (row < nr) {
                b0 = (int)(rp[rs + row] - ps);
                e0 = (int)(rp[rs + row + 1] - ps);
            }
            int ci[PPT];
            VT vv[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int t = tid + q * BLOCK;
                if (t < cnt) {
                    ci[q] = col[ps + t];
                    vv[q] = val[ps + t];
                }
            }
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int t = tid + q * BLOCK;
                if (t < cnt) prod[t] = to_a(vv[q], AT(0)) * to_a(x[ci[q]], AT(0));
            }
            __syncthreads();
            AT s = AT(0);
            for (int k = b0 + lane; k < e0; k += tpr) s += prod[k];
            for (int o = tpr >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (row < nr && lane == 0) epi(rs + row, (double)s, false, 0);
            __syncthreads();
        } else {
            const int lid = -1 - item.x;
            const int64_t r = lrow[lid];
            const int64_t p0 = rp[r] + (int64_t)item.y * CH;
            const int64_t p1 = min(p0 + (int64_t)CH, rp[r + 1]);
            const int cnt = (int)(p1 - p0);
            AT s = AT(0);
            for (int base = 0; base < cnt; base += PPT * BLOCK) {
                int ci[PPT];
                VT vv[PPT];
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const int t = base + tid + q * BLOCK;
                    if (t < cnt) {
                        ci[q] = col[p0 + t];
                        vv[q] = val[p0 + t];
                    }
                }
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const int t = base + tid + q * BLOCK;
                    if (t < cnt) s += to_a(vv[q], AT(0)) * to_a(x[ci[q]], AT(0));
                }
            }
            s = block_sum(s, sha);
            if (tid == 0) st_dev(&lpart[it], (double)s);
            if (last_block(&ltk[lid], (uint32_t)lnch[lid], &s_last)) {
                if (tid == 0) {
                    const int f = lfirst[lid], nc = lnch[lid];
                    double tot = 0.0;
                    for (int q = 0; q < nc; ++q) tot += ld_dev(&lpart[f + q]);
                    epi(r, tot, true, lid);
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace lz
