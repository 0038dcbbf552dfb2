// The stream-ordered solve shared by the entry points that enqueue a whole
// solve without waiting for the device.  Nothing here is part of the C ABI.
#pragma once

#include "../../include/lanczos_topk.h"
#include "lz_internal.h"

namespace lz {

// Checks the arguments of a stream-ordered solve (those of
// lanczos_topk_async) and fills the effective options, the plan and the
// restart budget.  Returns LZ_OK or the lz_status to return.
int check_async(const int64_t* rowptr, const int32_t* col, const void* val, int64_t n, int64_t nnz, int32_t K,
                int32_t m, int32_t precision, const double* out_vals, const double* out_vecs,
                const lz_options* opt, lz_options* o, Plan* p, int* budget);

// Enqueues the whole solve on s (no host synchronisation).  ws: device
// memory of at least p.bytes, or null to allocate it stream-ordered.
int run_solve_async(Plan p, Csr a, const lz_options& o, int budget, hipStream_t s, double* out_vals,
                    double* out_vecs, void* d_report, void* ws);

}  // namespace lz
