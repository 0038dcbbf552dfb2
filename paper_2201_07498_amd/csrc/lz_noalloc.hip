// lanczos_topk_noalloc: the stream-ordered solve of lanczos_topk_async with
// its workspace in a fixed device array of the library, for callers that
// cannot allocate device memory (code under hipGraph capture, serving loops,
// harnesses that forbid allocation).  Same kernels, same launch sequence.
//
// The array lives in the code object (`scratch`, LZ_NOALLOC_SCRATCH_BYTES),
// so every GPU the library runs on holds its own copy until the process
// ends.  Its device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and is passed to the kernels like any
// workspace; the symbol itself is never handed to a kernel or a copy.  Every
// call on a device uses the same array: calls that overlap on one device
// (different streams, or threads without ordering) race.  Nothing in the
// array needs clearing between calls: the solve's first kernels write every
// location it later reads (state reset, tile tables, start vector and the
// working vector), as with a caller workspace of uninitialised memory.
#include <mutex>

#include "../../include/lanczos_topk.h"
#include "lz_solve.h"

namespace lz {
namespace {

__device__ __align__(256) unsigned char scratch[LZ_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the
// device's first call), or null on failure.
void* scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace lz

using namespace lz;

extern "C" {

size_t lanczos_topk_noalloc_max_bytes(void) { return (size_t)LZ_NOALLOC_SCRATCH_BYTES; }

int lanczos_topk_noalloc(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val, int64_t n,
                         int64_t nnz, int32_t K, int32_t m, int32_t precision, void* stream, double* out_vals,
                         double* out_vecs, const lz_options* opt, lz_report* d_report) {
    lz_options o;
    Plan p;
    int budget = 0;
    const int rc = check_async(csr_rowptr, csr_col, csr_val, n, nnz, K, m, precision, out_vals, out_vecs, opt, &o,
                               &p, &budget);
    if (rc != LZ_OK) return rc;
    if (o.workspace) return LZ_ERR_INVALID_ARG;
    if (p.bytes > (size_t)LZ_NOALLOC_SCRATCH_BYTES) return LZ_ERR_TOO_LARGE;
    void* ws = scratch_ptr();
    if (!ws) return LZ_ERR_HIP;
    return run_solve_async(p, Csr{csr_rowptr, csr_col, csr_val, n, nnz}, o, budget, (hipStream_t)stream, out_vals,
                           out_vecs, d_report, ws);
}

}  // extern "C"
