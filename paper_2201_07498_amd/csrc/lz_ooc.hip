// Host-resident matrices: slab planning, device buffers and the copy stream
// (the passes themselves are ooc_pass in lz_ooc.h).
#include <algorithm>
#include <vector>

#include "lz_ooc.h"
#include "lz_spmv.h"

namespace lz {

namespace {
// Streams and events of the host-resident solves, created on first use per
// host thread and device and kept for the process: a freshly created pair of
// streams has been measured to block the host thread for milliseconds during
// its first few dozen copies and cross-stream waits.
struct StreamSet {
    hipStream_t ks = nullptr, cs = nullptr;
    hipEvent_t join = nullptr;
    hipEvent_t ready[2] = {nullptr, nullptr};
    hipEvent_t freed[2] = {nullptr, nullptr};
};
constexpr int MAX_DEVICES = 64;
thread_local StreamSet stream_sets[MAX_DEVICES];

hipError_t stream_set(StreamSet** out) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= MAX_DEVICES) return hipErrorInvalidDevice;
    StreamSet& S = stream_sets[d];
    if (!S.join) {
        StreamSet N;
        const unsigned ef = hipEventDisableTiming;
        if ((e = hipStreamCreateWithFlags(&N.ks, hipStreamNonBlocking)) == hipSuccess &&
            (e = hipStreamCreateWithFlags(&N.cs, hipStreamNonBlocking)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&N.ready[0], ef)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&N.ready[1], ef)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&N.freed[0], ef)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&N.freed[1], ef)) == hipSuccess &&
            (e = hipEventCreateWithFlags(&N.join, ef)) == hipSuccess) {
            S = N;
        } else {
            for (hipStream_t x : {N.ks, N.cs})
                if (x) (void)hipStreamDestroy(x);
            for (hipEvent_t x : {N.ready[0], N.ready[1], N.freed[0], N.freed[1], N.join})
                if (x) (void)hipEventDestroy(x);
            return e;
        }
    }
    *out = &S;
    return hipSuccess;
}
}  // namespace

hipError_t ooc_begin(Ooc& o, hipStream_t* s) {
    StreamSet* S = nullptr;
    hipError_t e = stream_set(&S);
    if (e != hipSuccess) return e;
    o.ks = S->ks;
    o.cs = S->cs;
    o.join = S->join;
    for (int i = 0; i < 2; ++i) {
        o.ready[i] = S->ready[i];
        o.freed[i] = S->freed[i];
    }
    if ((e = hipEventRecord(o.join, *s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(o.ks, o.join, 0)) != hipSuccess) return e;
    *s = o.ks;
    return hipSuccess;
}

hipError_t ooc_end(Ooc& o, hipStream_t user) {
    hipError_t e;
    if ((e = hipEventRecord(o.join, o.ks)) != hipSuccess) return e;
    return hipStreamWaitEvent(user, o.join, 0);
}

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
        for (int i = 0; i < 2; ++i)
            if ((e = hipEventRecord(o.freed[i], s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

void ooc_release(Ooc& o) {
    // The streams and events stay cached for the next solve on this thread.
    if (o.ks) (void)hipStreamSynchronize(o.ks);
    if (o.cs) (void)hipStreamSynchronize(o.cs);
    o.ks = o.cs = nullptr;
    o.join = nullptr;
    for (int i = 0; i < 2; ++i) {
        o.ready[i] = o.freed[i] = nullptr;
        if (o.scol[i]) (void)hipFree(o.scol[i]);
        if (o.sval[i]) (void)hipFree(o.sval[i]);
        o.scol[i] = nullptr;
        o.sval[i] = nullptr;
    }
    if (o.rcol) (void)hipFree(o.rcol);
    if (o.rval) (void)hipFree(o.rval);
    o.rcol = nullptr;
    o.rval = nullptr;
}

}  // namespace lz
