// Host-resident matrices: slab planning, device buffers and the copy stream
// (the passes themselves are ooc_pass in lz_ooc.h).
#include <algorithm>
#include <vector>

#include "lz_ooc.h"
#include "lz_spmv.h"

namespace lz {

hipError_t ooc_prepare(Plan& p, const Bufs& b, Ooc& o, int64_t slab_nnz, int64_t resident_nnz, hipStream_t s) {
    hipError_t e;
    // Status of the row-pointer checks and the tile table built from them.
    std::vector<int32_t> ob((size_t)p.n_tiles + 1);
    int32_t status = 0;
    if ((e = hipMemcpyAsync(&status, &b.st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(ob.data(), b.ob, ob.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    o.tb.assign(1, 0);
    o.eb.assign(1, 0);
    o.nres = 0;
    o.next = 0;
    o.validated = false;
    o.streamed = 0;
    p.g_slab = 8;
    // Bad row pointers: no slabs; every later kernel sees the status and returns.
    if (status != 0) return hipSuccess;

    // Slabs: greedy runs of whole tiles of at most slab_nnz entries.  Tile t
    // starts at entry t*TILE - ob[t] (the items before it are its entries and
    // the row ends of rows 0 .. ob[t]-1); a tile holds at most TILE entries.
    auto ent = [&](int64_t t) -> int64_t { return t >= p.n_tiles ? p.nnz : t * TILE - ob[t]; };
    for (int64_t t = 0; t < p.n_tiles;) {
        int64_t u = t + 1;
        while (u < p.n_tiles && ent(u + 1) - ent(t) <= slab_nnz) ++u;
        o.tb.push_back(u);
        o.eb.push_back(ent(u));
        t = u;
    }
    const int ns = o.nslab();
    for (int k = 0; k < ns; ++k)
        if (o.eb[k + 1] < o.eb[k] || o.eb[k + 1] - o.eb[k] > slab_nnz) return hipErrorInvalidValue;
    if (o.eb[ns] != p.nnz) return hipErrorInvalidValue;
    while (o.nres < ns && o.eb[o.nres + 1] <= resident_nnz) ++o.nres;

    // One grid for every slab launch: enough wavefronts for the largest slab,
    // and the alpha partials of all slabs (ns * grid) fit the partial buffer.
    int64_t maxt = 0, maxe = 0;
    for (int k = 0; k < ns; ++k) {
        maxt = std::max(maxt, o.tb[k + 1] - o.tb[k]);
        if (k >= o.nres) maxe = std::max(maxe, o.eb[k + 1] - o.eb[k]);
    }
    int64_t g = std::min<int64_t>(p.g_tile, (maxt + WAVES - 1) / WAVES);
    g = (g + 7) / 8 * 8;
    const int64_t cap = (int64_t)std::max(std::max(p.g_tile, p.g_dense), 2048) * 64;
    if ((int64_t)ns * g > cap) g = cap / ns / 8 * 8;
    if (g < 8) return hipErrorInvalidValue;
    p.g_slab = (int32_t)g;

    // Resident slabs: one copy, on the solve's stream.
    const int64_t eres = o.eb[o.nres];
    if (eres > 0) {
        if ((e = hipMalloc((void**)&o.rcol, (size_t)eres * 4)) != hipSuccess) return e;
        if ((e = hipMalloc((void**)&o.rval, (size_t)eres * o.vb)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(o.rcol, o.hcol, (size_t)eres * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(o.rval, o.hval, (size_t)eres * o.vb, hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        o.streamed += eres * (int64_t)(4 + o.vb);
    }
    // Staging buffers and the copy stream for the others.
    if (o.nres < ns) {
        const size_t me = (size_t)std::max<int64_t>(maxe, 1);
        for (int i = 0; i < 2; ++i) {
            if ((e = hipMalloc((void**)&o.scol[i], me * 4)) != hipSuccess) return e;
            if ((e = hipMalloc((void**)&o.sval[i], me * o.vb)) != hipSuccess) return e;
        }
        if ((e = hipStreamCreateWithFlags(&o.cs, hipStreamNonBlocking)) != hipSuccess) return e;
        for (int i = 0; i < 2; ++i) {
            if ((e = hipEventCreateWithFlags(&o.ready[i], hipEventDisableTiming)) != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&o.freed[i], hipEventDisableTiming)) != hipSuccess) return e;
            if ((e = hipEventRecord(o.freed[i], s)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

void ooc_release(Ooc& o) {
    if (o.cs) {
        (void)hipStreamSynchronize(o.cs);
        (void)hipStreamDestroy(o.cs);
        o.cs = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        if (o.ready[i]) (void)hipEventDestroy(o.ready[i]);
        if (o.freed[i]) (void)hipEventDestroy(o.freed[i]);
        if (o.scol[i]) (void)hipFree(o.scol[i]);
        if (o.sval[i]) (void)hipFree(o.sval[i]);
        o.ready[i] = o.freed[i] = nullptr;
        o.scol[i] = nullptr;
        o.sval[i] = nullptr;
    }
    if (o.rcol) (void)hipFree(o.rcol);
    if (o.rval) (void)hipFree(o.rval);
    o.rcol = nullptr;
    o.rval = nullptr;
}

}  // namespace lz
