// Host-resident matrices, for matrices whose entries do not fit in device
// memory.  The paper reaches such out-of-core matrices through unified memory
// paging (Sec. III-B) and measures them with only part of the input on the
// GPU at a time (Sec. IV-B); here the transfers are explicit.
//
// The row pointers (8 bytes per row) are copied to the device once; the
// column indices and values (4 + value bytes per entry) stay in pinned host
// memory.  The matrix is cut into slabs of whole SpMV tiles, so a slab is a
// contiguous range of entries and the split-row machinery of the tiles joins
// rows that cross a slab boundary exactly as it joins rows that cross a tile
// boundary.  Every pass over the matrix (each Lanczos-step SpMV, the residual
// product of the report) walks the slabs in order:
//   * the leading `nres` slabs stay on the device after their first copy
//     (the share of device memory the caller grants the matrix);
//   * the others are copied into two staging buffers in turn on a copy
//     stream, so the copy of slab k + 1 overlaps the kernel of slab k, and the
//     first streamed slab of the next pass is copied while the
//     orthogonalisation kernels of the current step run;
//   * the first pass checks every column index before the slab's kernel
//     gathers through it.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/lanczos_topk.h"
#include "lz_internal.h"

namespace lz {

struct Ooc {
    const int32_t* hcol = nullptr;   // pinned host arrays of the caller, nnz entries
    const char* hval = nullptr;
    size_t vb = 0;                   // bytes per value
    int64_t n = 0;
    std::vector<int64_t> tb;         // slab k: tiles [tb[k], tb[k+1])
    std::vector<int64_t> eb;         //         entries [eb[k], eb[k+1])
    int nres = 0;                    // slabs 0 .. nres-1 stay on the device
    int32_t* rcol = nullptr;         // resident entries [0, eb[nres])
    char* rval = nullptr;
    int32_t* scol[2] = {nullptr, nullptr};   // staging buffers of the streamed slabs
    char* sval[2] = {nullptr, nullptr};
    hipStream_t ks = nullptr;        // compute stream of the solve (default priority)
    hipStream_t cs = nullptr;        // copy stream (default priority)
    hipEvent_t join = nullptr;       // orders the compute stream after the caller's stream and back
    hipEvent_t ready[2] = {nullptr, nullptr};   // staging buffer i holds its slab
    hipEvent_t freed[2] = {nullptr, nullptr};   // the kernel reading staging buffer i is done
    int next = 0;                    // staging buffer of the next streamed slab
    bool validated = false;          // every column index has been checked
    int64_t streamed = 0;            // host-to-device bytes enqueued after the resident copy

    int nslab() const { return (int)tb.size() - 1; }
};

// Pointer p shifted back by e0 elements of `bytes` each, so that entry e of
// the matrix is element e of the result for the entries a buffer holds.
template <class T>
inline T* entry_base(T* p, int64_t e0, size_t bytes) {
    return (T*)((uintptr_t)p - (uintptr_t)e0 * (uintptr_t)bytes);
}

// One pass over a host-resident matrix on stream s: for slab k = 0 .. nslab-1
// in order, launch(col, val, tb, te, k, nslab) once the slab's entries are on
// the device, with col/val indexed by matrix entry.
template <class L>
hipError_t ooc_pass(Ooc& o, State* st, hipStream_t s, L&& launch) {
    const int ns = o.nslab();
    hipError_t e = hipSuccess;
    for (int k = 0; k < ns; ++k) {
        const int64_t e0 = o.eb[k], e1 = o.eb[k + 1];
        const int32_t* c;
        const char* v;
        int i = -1;
        if (k < o.nres) {
            c = o.rcol;
            v = o.rval;
        } else {
            i = o.next;
            o.next ^= 1;
            if ((e = hipStreamWaitEvent(o.cs, o.freed[i], 0)) != hipSuccess) return e;
            if (e1 > e0) {
                if ((e = hipMemcpyAsync(o.scol[i], o.hcol + e0, (size_t)(e1 - e0) * 4, hipMemcpyHostToDevice,
                                        o.cs)) != hipSuccess)
                    return e;
                if ((e = hipMemcpyAsync(o.sval[i], o.hval + (size_t)e0 * o.vb, (size_t)(e1 - e0) * o.vb,
                                        hipMemcpyHostToDevice, o.cs)) != hipSuccess)
                    return e;
                o.streamed += (e1 - e0) * (int64_t)(4 + o.vb);
            }
            if ((e = hipEventRecord(o.ready[i], o.cs)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, o.ready[i], 0)) != hipSuccess) return e;
            c = entry_base((const int32_t*)o.scol[i], e0, 4);
            v = entry_base((const char*)o.sval[i], e0, o.vb);
        }
        if (!o.validated) launch_validate_cols(st, c, e0, e1, o.n, s);
        launch(c, (const void*)v, o.tb[k], o.tb[k + 1], k, ns);
        if (i >= 0 && (e = hipEventRecord(o.freed[i], s)) != hipSuccess) return e;
    }
    o.validated = true;
    return hipGetLastError();
}

// A host-resident matrix of one solve and its streaming state.
struct HostCsr {
    int64_t slab_nnz = 0;       // entries per streamed slab (>= TILE)
    int64_t resident_nnz = 0;   // leading entries that may stay on the device
    Ooc ooc;
};

// The launch sequence of one solve (arguments already checked).  With hc
// non-null, a.rowptr is a host array, a.col/a.val are unused and the entries
// come from hc->ooc.
int run_solve(Plan p, Csr a, const lz_options& o, hipStream_t s, double* out_vals, double* out_vecs,
              lz_report* report, HostCsr* hc);

// The solve runs on a compute stream of its own (cached per host thread and
// device with the copy stream and the events), ordered after the caller's
// stream, so that the copy and compute streams are both created streams
// whatever stream the caller passes.  *s becomes that stream.
hipError_t ooc_begin(Ooc& o, hipStream_t* s);
// Makes the caller's stream wait for the compute stream.
hipError_t ooc_end(Ooc& o, hipStream_t user);

// Plans the slabs from the device tile table and sets up the buffers and the
// copy stream; copies the resident slabs.  slab_nnz >= TILE.
hipError_t ooc_prepare(Plan& p, const Bufs& b, Ooc& o, int64_t slab_nnz, int64_t resident_nnz, hipStream_t s);
// Waits for both streams and frees what ooc_begin and ooc_prepare allocated.
void ooc_release(Ooc& o);

}  // namespace lz
