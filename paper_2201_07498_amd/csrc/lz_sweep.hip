// Sweep-block copy of the relabelled matrix (Algorithm 1, the SpMV line, on
// large power-law matrices): the setup kernels that cut the rows into sweep
// blocks and store each block's entries in column order.
//
// Why: after the hub-first relabelling the gathers of x in row order land on
// random lines of a vector far larger than L2, one 128-byte line per
// gathered entry.  A wavefront that walks a block's entries in column order
// gathers x from low to high addresses, and all wavefronts of the chip do
// so at about the same pace, so the lines one XCD pulls in are reused by its
// other wavefronts before they leave L2.  The row sums are then accumulated
// in LDS (one slot per row of the block) instead of in row order.
//
// Build (all on the device, stream-ordered): the block table (first owned
// row and first entry of every block), one segmented radix sort of the
// relabelled column indices with the entry positions as values (rocPRIM,
// one segment per block, keys sorted on the bits above the line offset so
// that entries of one line keep their row order), then the rows within the
// block and the values, gathered by the sorted positions.
#include <cstring>

#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "../../include/lanczos_topk.h"
#include "lz_spmv.h"

namespace lz {

namespace {

// One workgroup per segment through all radix passes, no partitioning of
// the segments by size: rocPRIM's partitioned path reads segment counts back
// to the host, which a stream-ordered solve cannot do.
using SortConfig = rocprim::segmented_radix_sort_config<8, rocprim::kernel_config<256, 16>,
                                                        rocprim::DisabledWarpSortConfig, false>;

hipError_t sort_blocks(void* tmp, size_t& bytes, const uint32_t* keys_in, uint32_t* keys_out, uint32_t* src,
                       int64_t nnz, int64_t nb, const int64_t* begin, int bit0, int bit1, hipStream_t s) {
    return rocprim::segmented_radix_sort_pairs<SortConfig>(
        tmp, bytes, keys_in, keys_out, rocprim::counting_iterator<uint32_t>(0u), src, (unsigned int)nnz,
        (unsigned int)nb, begin, begin + 1, (unsigned int)bit0, (unsigned int)bit1, s);
}

// Block table: ob[b] = first row whose end item lies at or after b * items
// (n if none), e[b] = first entry of block b.  When the device did
// not choose the sweep-block copy every block is empty (e = 0), so the sort
// that follows has nothing to do.
__global__ __launch_bounds__(BLOCK) void k_sw_blocks(const State* st, const int64_t* __restrict__ rp, int64_t n,
                                                     int64_t nnz, int64_t nb, int64_t items, int32_t* ob,
                                                     int64_t* e) {
    const bool on = st->status == 0 && st->reordered && st->packed == PACK_SWEEP;
    for (int64_t b = (int64_t)blockIdx.x * BLOCK + threadIdx.x; b <= nb; b += (int64_t)gridDim.x * BLOCK) {
        if (!on) {
            ob[b] = 0;
            e[b] = 0;
            continue;
        }
        const int64_t target = b * items;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (rp[mid + 1] + SW_W * mid >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        ob[b] = (int32_t)lo;
        e[b] = lo < n ? max(rp[lo], target - SW_W * lo) : nnz;
    }
}

constexpr int SWF_WAVES = 4;

// Rows within the block and values of the column-sorted entries: entry p of
// block b came from position src[p] of the row-ordered copy; its row is the
// last of the block's rows (staged in LDS as starts relative to the block)
// that starts at or before that position.  One wavefront per block.
template <class VT, int ROWS>
__global__ __launch_bounds__(SWF_WAVES * 64) void k_sw_fill(const State* st, const int64_t* __restrict__ rp,
                                                            const VT* __restrict__ val2, int64_t nb,
                                                            const int32_t* __restrict__ ob,
                                                            const int64_t* __restrict__ e,
                                                            const uint32_t* __restrict__ src,
                                                            uint16_t* __restrict__ rl, VT* __restrict__ val) {
    __shared__ int32_t srow[SWF_WAVES][ROWS + 2];
    if (st->status != 0 || !st->reordered || st->packed != PACK_SWEEP) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t* s = srow[w];
    for (int64_t b = (int64_t)blockIdx.x * SWF_WAVES + w; b < nb; b += (int64_t)gridDim.x * SWF_WAVES) {
        const int64_t r0 = ob[b], e0 = e[b];
        const int nown = ob[b + 1] - (int32_t)r0;
        const int cnt = (int)(e[b + 1] - e0);
        if (cnt <= 0) continue;
        for (int i = lane; i <= nown; i += 64) s[i] = (int32_t)max<int64_t>(rp[r0 + i] - e0, -1);
        wave_sync();
        for (int k = lane; k < cnt; k += 64) {
            const int64_t p = e0 + k;
            const uint32_t from = src[p];
            const int loc = (int)((int64_t)from - e0);
            int lo = 0;
#pragma unroll
            for (int step = ROWS; step > 0; step >>= 1)
                if (lo + step <= nown && s[lo + step] <= loc) lo += step;
            rl[p] = (uint16_t)lo;
            val[p] = val2[from];
        }
        wave_sync();
    }
}

}  // namespace

bool sweep_applies(int64_t n, int64_t nnz, int prec, int request) {
    if (request == LZ_SWEEP_OFF || n < 2 || nnz <= 0) return false;
    // The sort counts entries and blocks in 32 bits.
    if (nnz >= (int64_t(1) << 32) - 1) return false;
    if (request == LZ_SWEEP_ON) return true;
    return n >= SWEEP_AUTO_MIN_N && (uint64_t)n * storage_bytes(prec) >= SWEEP_AUTO_MIN_X_BYTES;
}

size_t sweep_sort_bytes(int64_t nnz, int64_t nb) {
    size_t bytes = 0;
    if (sort_blocks(nullptr, bytes, nullptr, nullptr, nullptr, nnz, nb, nullptr, 0, 32, nullptr) == hipSuccess &&
        bytes > 0)
        return bytes;
    // No device to ask (the sort's size query looks up the GPU): its two
    // double buffers plus slack; a solve checks the real size before use.
    return (size_t)nnz * 8 + ((size_t)1 << 20);
}

hipError_t launch_sweep_setup(const Plan& p, const Bufs& b, hipStream_t s) {
    if (!p.sweep) return hipSuccess;
    size_t need = 0;
    hipError_t err = sort_blocks(nullptr, need, nullptr, nullptr, nullptr, p.nnz, p.sw_nb, nullptr, p.sw_bit0,
                                 p.sw_bit1, s);
    if (err != hipSuccess) return err;
    if (need > p.sw_sort_bytes) return hipErrorInvalidValue;
    const int gb = (int)std::min<int64_t>((p.sw_nb + BLOCK) / BLOCK, 1024);
    hipLaunchKernelGGL(k_sw_blocks, dim3(gb), dim3(BLOCK), 0, s, b.st, b.rp2, p.n, p.nnz, p.sw_nb, p.sw_items,
                       b.swob, b.swe);
    size_t bytes = p.sw_sort_bytes;
    err = sort_blocks(b.swtmp, bytes, (const uint32_t*)b.col2, (uint32_t*)b.swcol, b.swsrc, p.nnz, p.sw_nb, b.swe,
                      p.sw_bit0, p.sw_bit1, s);
    if (err != hipSuccess) return err;
    const int gf = (int)std::min<int64_t>((p.sw_nb + SWF_WAVES - 1) / SWF_WAVES, 2048);
    switch (p.prec) {
        case 0:
            hipLaunchKernelGGL((k_sw_fill<double, sweep_rows(0)>), dim3(gf), dim3(SWF_WAVES * 64), 0, s, b.st, b.rp2,
                               (const double*)b.val2, p.sw_nb, b.swob, b.swe, b.swsrc, b.swrl, (double*)b.swval);
            break;
        case 1:
            hipLaunchKernelGGL((k_sw_fill<float, sweep_rows(1)>), dim3(gf), dim3(SWF_WAVES * 64), 0, s, b.st, b.rp2,
                               (const float*)b.val2, p.sw_nb, b.swob, b.swe, b.swsrc, b.swrl, (float*)b.swval);
            break;
        default:
            hipLaunchKernelGGL((k_sw_fill<uint16_t, sweep_rows(2)>), dim3(gf), dim3(SWF_WAVES * 64), 0, s, b.st, b.rp2,
                               (const uint16_t*)b.val2, p.sw_nb, b.swob, b.swe, b.swsrc, b.swrl,
                               (uint16_t*)b.swval);
            break;
    }
    return hipGetLastError();
}

}  // namespace lz
