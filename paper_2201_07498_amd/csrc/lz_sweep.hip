// Sweep-block copy of the relabelled matrix (Algorithm 1, the SpMV line, on
// large power-law matrices): the setup kernels that cut the rows into sweep
// blocks and store each block's entries in column order.
//
// Why: in row order the 64 gathers of one wavefront instruction fall on up
// to 64 different 128-byte lines of x, and beyond L2 each line costs a
// memory request.  A wavefront that walks a block's entries in column order
// gathers neighbouring columns in one instruction, which share lines, above
// all in the dense head of x where the hub-first relabelling put the most
// gathered columns.  (Measured at R-MAT scale 26, FP32: 1.02e9 -> 6.5e8
// read requests per SpMV at about the same L2 hit rate.)  The row sums are
// then accumulated in LDS (one slot per row of the block) instead of in row
// order.
//
// Build (all on the device, stream-ordered): the block table (first owned
// row and first entry of every block); the relabelling fill then writes each
// entry's row within its block and position within it (one 32-bit word, in
// row order); one segmented radix sort of the relabelled column indices with
// those words as values (rocPRIM, one segment per block, keys sorted on the
// bits above the line offset so that entries of one line keep their row
// order); then the rows and, gathered by the sorted positions, the values.
#include <cstring>

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "../../include/lanczos_topk.h"
#include "lz_spmv.h"

namespace lz {

namespace {

// One workgroup per segment through all radix passes, no partitioning of
// the segments by size: rocPRIM's partitioned path reads segment counts back
// to the host, which a stream-ordered solve cannot do.
using SortConfig = rocprim::segmented_radix_sort_config<8, rocprim::kernel_config<256, 16>,
                                                        rocprim::DisabledWarpSortConfig, false>;

hipError_t sort_blocks(void* tmp, size_t& bytes, const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* vin,
                       uint32_t* vout, int64_t nnz, int64_t nb, const int64_t* begin, int bit0, int bit1,
                       hipStream_t s) {
    return rocprim::segmented_radix_sort_pairs<SortConfig>(tmp, bytes, keys_in, keys_out, vin, vout,
                                                           (unsigned int)nnz, (unsigned int)nb, begin, begin + 1,
                                                           (unsigned int)bit0, (unsigned int)bit1, s);
}

// Block table: ob[b] = first row whose end item lies at or after b * items
// (n if none), e[b] = first entry of block b.  When the device did
// not choose the sweep-block copy every block is empty (e = 0), so the sort
// that follows has nothing to do.
__global__ __launch_bounds__(BLOCK) void k_sw_blocks(const State* st, const int64_t* __restrict__ rp, int64_t n,
                                                     int64_t nnz, int64_t nb, int64_t items, int32_t* ob,
                                                     int64_t* e, uint32_t* queue) {
    const bool on = st->status == 0 && st->reordered && st->packed == PACK_SWEEP;
    if (blockIdx.x == 0 && threadIdx.x < 8) queue[threadIdx.x] = 0u;
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

// Measured on MI355X, R-MAT 26 FP32 (grid / slices per block / entries per
// thread in flight -> fill ms): 1024/32/1 22.6, 1024/8/8 17.2, 512/16/8
// 15.4, 256/16/8 17.2, 512/32/4 22.8, 1024/64/2 36.0, 256/8/16 12.3,
// 256/8/32 12.4, 256/4/16 12.3, 512/8/16 13.1, 128/8/32 20.5.  The first
// form, one wavefront per block with the rows found by binary search in LDS,
// took 27.9 ms.
constexpr int SWF_THREADS = 256;
constexpr int SWF_GRID = 256;
constexpr int SWF_SLICES = 8;         // work items per block
constexpr int SWF_U = 16;             // entries per thread in flight

// Rows within the block and values of the column-sorted entries: the sorted
// payload of entry p of block b holds its row within the block and its
// position in the block's row-ordered entries, from which its value is
// gathered.  Those gathers fall anywhere in the block (up to 512 KB of values
// in FP32, 2 MB in FP64).  So XCD x (workgroup i runs on XCD i mod 8) takes
// the blocks b = x mod 8 in order, and its workgroups draw the slices of
// those blocks from one counter per XCD: at any time an XCD works on one or
// two blocks, whose values stay in its L2 while they are gathered.  The
// payload stream and the outputs bypass L2.  Every entry's outputs depend on
// the entry alone, so the order in which slices are drawn does not matter.
// A workgroup draws its next slice before working on the current one, and
// each thread keeps SWF_U entries in flight, so the chain of dependent loads
// (payload, then value) is paid once per SWF_U entries.
template <class VT>
__global__ __launch_bounds__(SWF_THREADS) void k_sw_fill(const State* st, const VT* __restrict__ val2, int64_t nb,
                                                         const int64_t* __restrict__ e,
                                                         const uint32_t* __restrict__ src,
                                                         uint16_t* __restrict__ rl, VT* __restrict__ val,
                                                         uint32_t* queue) {
    __shared__ uint32_t s_item[2];
    if (st->status != 0 || !st->reordered || st->packed != PACK_SWEEP) return;
    constexpr uint32_t POSMASK = (1u << SW_POSBITS) - 1u;
    const uint32_t xcd = blockIdx.x & 7u;
    const int64_t nbx = (nb - xcd + 7) / 8;      // blocks of this XCD
    const int64_t items = nbx * SWF_SLICES;
    if (threadIdx.x == 0)
        s_item[0] = __hip_atomic_fetch_add(queue + xcd, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (int it = 0;; it ^= 1) {
        const int64_t item = s_item[it];
        if (item >= items) break;
        if (threadIdx.x == 0)
            s_item[it ^ 1] = __hip_atomic_fetch_add(queue + xcd, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t b = xcd + 8 * (item / SWF_SLICES), slice = item % SWF_SLICES;
        const int64_t e0 = e[b], cnt = e[b + 1] - e0;
        const int64_t k0 = cnt * slice / SWF_SLICES, k1 = cnt * (slice + 1) / SWF_SLICES;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += SWF_THREADS * SWF_U) {
            uint32_t w[SWF_U];
#pragma unroll
            for (int q = 0; q < SWF_U; ++q)
                w[q] = __builtin_nontemporal_load(src + e0 + min<int64_t>(k + q * SWF_THREADS, k1 - 1));
            VT v[SWF_U];
#pragma unroll
            for (int q = 0; q < SWF_U; ++q) v[q] = val2[e0 + (w[q] & POSMASK)];
#pragma unroll
            for (int q = 0; q < SWF_U; ++q) {
                const int64_t kq = k + q * SWF_THREADS;
                if (kq < k1) {
                    __builtin_nontemporal_store((uint16_t)(w[q] >> SW_POSBITS), rl + e0 + kq);
                    __builtin_nontemporal_store(v[q], val + e0 + kq);
                }
            }
        }
        __syncthreads();                         // the next item is visible; this one is no longer read
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
    if (sort_blocks(nullptr, bytes, nullptr, nullptr, nullptr, nullptr, nnz, nb, nullptr, 0, 32, nullptr) ==
            hipSuccess &&
        bytes > 0)
        return bytes;
    // No device to ask (the sort's size query looks up the GPU): its two
    // double buffers plus slack; a solve checks the real size before use.
    return (size_t)nnz * 8 + ((size_t)1 << 20);
}

void launch_sweep_blocks(const Plan& p, const Bufs& b, hipStream_t s) {
    if (!p.sweep) return;
    const int gb = (int)std::min<int64_t>((p.sw_nb + BLOCK) / BLOCK, 1024);
    hipLaunchKernelGGL(k_sw_blocks, dim3(gb), dim3(BLOCK), 0, s, b.st, b.rp2, p.n, p.nnz, p.sw_nb, p.sw_items,
                       b.swob, b.swe, b.swq);
}

hipError_t launch_sweep_sort(const Plan& p, const Bufs& b, hipStream_t s) {
    if (!p.sweep) return hipSuccess;
    size_t need = 0;
    hipError_t err = sort_blocks(nullptr, need, nullptr, nullptr, nullptr, nullptr, p.nnz, p.sw_nb, nullptr,
                                 p.sw_bit0, p.sw_bit1, s);
    if (err != hipSuccess) return err;
    if (need > p.sw_sort_bytes) return hipErrorInvalidValue;
    size_t bytes = p.sw_sort_bytes;
    err = sort_blocks(b.swtmp, bytes, (const uint32_t*)b.col2, (uint32_t*)b.swcol, b.swvin, b.swsrc, p.nnz,
                      p.sw_nb, b.swe, p.sw_bit0, p.sw_bit1, s);
    if (err != hipSuccess) return err;
    switch (p.prec) {
        case 0:
            hipLaunchKernelGGL(k_sw_fill<double>, dim3(SWF_GRID), dim3(SWF_THREADS), 0, s, b.st,
                               (const double*)b.val2, p.sw_nb, b.swe, b.swsrc, b.swrl, (double*)b.swval, b.swq);
            break;
        case 1:
            hipLaunchKernelGGL(k_sw_fill<float>, dim3(SWF_GRID), dim3(SWF_THREADS), 0, s, b.st,
                               (const float*)b.val2, p.sw_nb, b.swe, b.swsrc, b.swrl, (float*)b.swval, b.swq);
            break;
        default:
            hipLaunchKernelGGL(k_sw_fill<uint16_t>, dim3(SWF_GRID), dim3(SWF_THREADS), 0, s, b.st,
                               (const uint16_t*)b.val2, p.sw_nb, b.swe, b.swsrc, b.swrl, (uint16_t*)b.swval,
                               b.swq);
            break;
    }
    return hipGetLastError();
}

}  // namespace lz
