// CSR SpMV core over merge-path tiles (Algorithm 1, the SpMV line), shared by
// the Lanczos step and the standalone SpMV.
//
// Walk the matrix as one sequence of items: the entries of row 0, an end
// marker for row 0, the entries of row 1, its end marker, and so on
// (nnz + n items; entry p of row r is item p + r, the end of row r is item
// rowptr[r+1] + r).  Tile t is items [t*TILE, (t+1)*TILE), one tile per
// wavefront at a time, so a tile holds at most TILE entries plus row ends
// whatever the row lengths (long rows, empty rows).  Row r is owned by the
// tile holding its end marker; tile t owns rows ob[t] .. ob[t+1]-1 and its
// entries are [t*TILE - ob[t], (t+1)*TILE - ob[t+1]).  A tile
//   * loads its col/val entries, gathers x and keeps the products in its
//     LDS slice;
//   * sums its owned rows: rows of up to LONGR entries by one lane each,
//     longer ones by the whole wavefront;
//   * may hold a head piece (its first owned row began in an earlier tile)
//     and a tail piece (row ob[t+1] continues into later tiles).
// A row whose first entry lies in tile t1 and whose end lies in tile t2 > t1
// has tail pieces in t1..t2-1 and the head piece in t2.  Every piece is
// published device-coherently and counted on the owner's ticket; the last
// piece to arrive adds all of them in tile order, so the row sum does not
// depend on which wavefront finishes last.
//
// The epilogue is four callbacks, all called by one lane:
//   pre(r)       a value the row epilogue needs (e.g. an entry of another
//                vector), loaded for the first 64 owned rows together with
//                the tile's entries;
//   row(r, s, p) owned row r with its whole sum s and p = pre(r);
//   piece(r, s)  one piece of a split row (for sums that are linear in the
//                row sum, such as alpha);
//   fin(r, s)    a split row's whole sum, from the finalising wavefront.
#pragma once

#include "lz_device.h"

namespace lz {

constexpr int WAVES = BLOCK / 64;
constexpr int TP = TILE / 64;          // tile entries per lane
constexpr int LONGR = 64;              // rows longer than this are summed by the whole wavefront

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

// Tile of item i, clamped so that malformed input cannot index outside the
// tile tables.
__device__ __forceinline__ int64_t item_tile(int64_t i, int64_t n_tiles) {
    const int64_t t = i / TILE;
    return t < 0 ? 0 : (t >= n_tiles ? n_tiles - 1 : t);
}
// Owner tile of row r (the tile of its end marker).
__device__ __forceinline__ int64_t row_owner(const int64_t* rp, int64_t r, int64_t n_tiles) {
    return item_tile(rp[r + 1] + r, n_tiles);
}

// Sum of p[b..e) in four interleaved chains, combined in a fixed order.
template <class AT>
__device__ __forceinline__ AT lds_sum(const AT* p, int b, int e) {
    AT s0 = AT(0), s1 = AT(0), s2 = AT(0), s3 = AT(0);
    int k = b;
    for (; k + 4 <= e; k += 4) {
        s0 += p[k];
        s1 += p[k + 1];
        s2 += p[k + 2];
        s3 += p[k + 3];
    }
    for (; k < e; ++k) s0 += p[k];
    return (s0 + s1) + (s2 + s3);
}

// Whole-wavefront sum of p[b..e): lane-strided partials, then the butterfly.
template <class AT>
__device__ __forceinline__ AT lds_wave_sum(const AT* p, int b, int e, int lane) {
    AT s = AT(0);
    for (int k = b + lane; k < e; k += 64) s += p[k];
    return wave_sum(s);
}

// Tiles handled by this wavefront out of tiles [tb, te) (all tiles, or one
// slab of a host-resident matrix): the range is split evenly over the eight
// XCDs (workgroup i runs on XCD i mod 8), so neighbouring tiles, which gather
// neighbouring parts of x in a banded matrix, share one L2.
struct TileRange {
    int64_t first, end, stride;
};
template <int NW = WAVES>
__device__ __forceinline__ TileRange wave_tiles(int64_t tb, int64_t te) {
    const int64_t xcd = blockIdx.x & 7, nb8 = gridDim.x >> 3;
    const int64_t nt = te - tb;
    const int64_t lo = tb + nt * xcd / 8, hi = tb + nt * (xcd + 1) / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)(blockIdx.x >> 3) * NW + wave;
    return {lo + w, hi, nb8 * NW};
}


// Adds the pieces of the split row r (tail pieces in tiles t1..t2-1, head
// piece in t2) in tile order; called by every lane of the finalising
// wavefront, returns the sum in all lanes.
__device__ __forceinline__ double split_total(const double* head, const double* tail, int64_t t1, int64_t t2,
                                              int lane) {
    double s = 0.0;
    for (int64_t i = t1 + lane; i < t2; i += 64) s += ld_dev(&tail[i]);
    s = wave_sum(s);
    return s + ld_dev(&head[t2]);
}

// Loads of the matrix streams (column indices and values), which every SpMV
// reads exactly once.  With NT they are non-temporal (the L2 does not keep
// them).  Measured on MI355X (SpMV per step, plain / non-temporal): FP64
// R-MAT 20 102.0 / 100.9 us, R-MAT 23 2.037 / 2.016 ms, R-MAT 26 24.4 /
// 23.7 ms; FP32 77.6 / 82.8 us, 1.552 / 1.577 ms, 18.8 / 19.0 ms.  So only
// the FP64 storage streams them non-temporally.
template <bool NT, class T> __device__ __forceinline__ T stream_load(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Bytes at the head of x gathered with ordinary loads (the L2 of one XCD);
// the rest non-temporally.  Measured on MI355X, step SpMV with and without:
// R-MAT scale 23 FP32 1542 -> 1375 us, scale 26 FP32 18.67 -> 18.37 ms and
// BF16 13.92 -> 13.63 ms; FP64 and R-MAT scale 20 unchanged.  A boundary at
// 1, 4 or 16 MB measured the same.
constexpr uint32_t GATHER_WARM_BYTES = 4u << 20;

// The products of one wavefront's share of stored entries [base, base+cnt)
// in LDS.  The 16 col/val loads of a lane go out together, then the 16
// gathers of x.  Lanes past the end re-read the last entry (same cache line),
// so every load is unconditional.  Row-ordered storage (slotbits = 0): entry
// base+k lands in pw[k], and lanes past the end land beyond cnt, never read.
// Column-sorted storage: each column word is (col << slotbits) | slot and the
// product lands in pw[slot], the entry's position in row order, so the row
// sums add the same values in the same order as for row-ordered storage
// (lanes past the end rewrite the last entry's product).  With CACHED, xs
// holds x[0..hn) in LDS and gathers of those entries read it.  With OFF32
// (every byte offset into x below 2^32), each load is a wave-uniform base in
// scalar registers plus a 32-bit per-lane offset, and the col and val loads
// of an entry share one offset; 64-bit per-lane addresses would otherwise take
// about half of the kernel's vector registers and limit its occupancy.
template <class VT, class AT, bool CACHED, bool OFF32>
__device__ __forceinline__ void tile_products(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                              const VT* __restrict__ x, const VT* xs, int hn, int64_t base, int cnt,
                                              int slotbits, AT* pw, int lane) {
    if (cnt <= 0) return;
    int ci[TP];
    VT vv[TP];
    constexpr bool NT = sizeof(VT) == 8;
    if constexpr (OFF32) {
        const char* cb = (const char*)(col + base);
        const char* vb = (const char*)(val + base);
#pragma unroll
        for (int q = 0; q < TP; ++q) {
            const uint32_t o = (uint32_t)min(q * 64 + lane, cnt - 1);
            ci[q] = stream_load<NT>((const int32_t*)(cb + o * 4u));
            vv[q] = stream_load<NT>((const VT*)(vb + o * (uint32_t)sizeof(VT)));
        }
    } else {
#pragma unroll
        for (int q = 0; q < TP; ++q) {
            const int64_t p = base + min(q * 64 + lane, cnt - 1);
            ci[q] = stream_load<NT>(col + p);
            vv[q] = stream_load<NT>(val + p);
        }
    }
    int sl[TP];
    const uint32_t smask = (1u << slotbits) - 1u;
#pragma unroll
    for (int q = 0; q < TP; ++q) {
        sl[q] = slotbits ? (int)((uint32_t)ci[q] & smask) : q * 64 + lane;
        ci[q] = (int)((uint32_t)ci[q] >> slotbits);
    }
#pragma unroll
    for (int q = 0; q < TP; ++q) {
        VT xv;
        // Entries of x past the first GATHER_WARM_BYTES are gathered
        // non-temporally: after the hub-first relabelling they are the rarely
        // used columns, and keeping their lines out of L2 leaves it to the
        // warm head of x.
        const bool warm = (uint32_t)ci[q] < GATHER_WARM_BYTES / (uint32_t)sizeof(VT);
        if constexpr (CACHED) {
            xv = ci[q] < hn ? xs[ci[q]] : (warm ? x[ci[q]] : __builtin_nontemporal_load(x + ci[q]));
        } else if constexpr (OFF32) {
            const VT* px = (const VT*)((const char*)x + (uint32_t)ci[q] * (uint32_t)sizeof(VT));
            xv = warm ? *px : __builtin_nontemporal_load(px);
        } else {
            xv = warm ? x[ci[q]] : __builtin_nontemporal_load(x + ci[q]);
        }
        pw[sl[q]] = to_a(vv[q], AT(0)) * to_a(xv, AT(0));
    }
}

// Row bounds of a tile's first 64 owned rows, pre() of those rows and the
// start of the row continuing past the tile; loaded with the tile's entries,
// so a tile waits for two rounds of requests (entries, then gathers) before
// its sums are written.
struct TileRows {
    int64_t t, t0, r_lo, r_hi, rb0, re0, rb_hi;
    double pv0;
    int cnt;
};
template <class Pre>
__device__ __forceinline__ TileRows tile_rows(const int64_t* __restrict__ rp, int64_t t, int64_t r_lo, int64_t r_hi,
                                              int64_t n, int64_t items, int lane, Pre&& pre) {
    TileRows q;
    q.t = t;
    q.r_lo = r_lo;
    q.r_hi = r_hi;
    q.t0 = t * TILE - r_lo;
    q.cnt = (int)(min<int64_t>((t + 1) * TILE, items) - r_hi - q.t0);
    const int64_t r_first = r_lo + lane;
    q.rb0 = 0;
    q.re0 = 0;
    q.pv0 = 0.0;
    if (r_first < r_hi) {
        q.rb0 = rp[r_first];
        q.re0 = rp[r_first + 1];
        q.pv0 = pre(r_first);
    }
    q.rb_hi = r_hi < n ? rp[r_hi] : 0;
    return q;
}

// Sums of one tile from its products pw[0..cnt) in row order: owned rows
// (one lane each up to LONGR entries, else the whole wavefront), then the
// head and tail pieces of split rows.
template <class AT, class Pre, class Row, class Piece, class Fin>
__device__ __forceinline__ void tile_sums(const TileRows& q, const AT* pw, const int64_t* __restrict__ rp, int64_t n,
                                          int64_t n_tiles, uint32_t* tk, double* head, double* tail, int lane,
                                          Pre&& pre, Row&& row, Piece&& piece, Fin&& fin) {
    const int64_t t = q.t, t0 = q.t0, r_lo = q.r_lo, r_hi = q.r_hi;
    const int cnt = q.cnt;
    // Owned rows, 64 at a time.
    const bool split_head = r_lo < r_hi && __shfl(q.rb0, 0, 64) < t0;
    double head_s = 0.0;
    for (int64_t base = r_lo; base < r_hi; base += 64) {
        const int64_t r = base + lane;
        const bool valid = r < r_hi;
        const bool first = base == r_lo;
        int b = 0, e = 0;
        double pv = 0.0;
        if (valid) {
            b = (int)(max(first ? q.rb0 : rp[r], t0) - t0);
            e = (int)((first ? q.re0 : rp[r + 1]) - t0);
            pv = first ? q.pv0 : pre(r);
        }
        const bool islong = valid && e - b > LONGR;
        AT s = (valid && !islong) ? lds_sum(pw, b, e) : AT(0);
        uint64_t mask = __ballot(islong);
        while (mask) {
            const int L = __builtin_ctzll(mask);
            mask &= mask - 1;
            const AT ss = lds_wave_sum(pw, __shfl(b, L, 64), __shfl(e, L, 64), lane);
            if (lane == L) s = ss;
        }
        if (valid) {
            if (split_head && r == r_lo) {
                head_s = (double)s;
                piece(r, head_s);
            } else {
                row(r, (double)s, pv);
            }
        }
    }
    // Head piece: publish, count, finish the row if it is the last piece.
    if (split_head) {
        if (lane == 0) st_dev(&head[t], head_s);
        const int64_t t1 = item_tile(rp[r_lo] + r_lo, n_tiles);
        if (last_wave(&tk[t], (uint32_t)(t - t1 + 1))) {
            const double tot = split_total(head, tail, t1, t, lane);
            if (lane == 0) fin(r_lo, tot);
        }
    }
    // Tail piece of the row that continues past this tile.
    if (r_hi < n) {
        const int64_t rb = q.rb_hi;
        if (rb < t0 + cnt) {
            const AT ss = lds_wave_sum(pw, (int)(max(rb, t0) - t0), cnt, lane);
            if (lane == 0) {
                piece(r_hi, (double)ss);
                st_dev(&tail[t], (double)ss);
            }
            const int64_t t1 = item_tile(rb + r_hi, n_tiles), t2 = row_owner(rp, r_hi, n_tiles);
            if (last_wave(&tk[t2], (uint32_t)(t2 - t1 + 1))) {
                const double tot = split_total(head, tail, t1, t2, lane);
                if (lane == 0) fin(r_hi, tot);
            }
        }
    }
}

// The workgroup's product buffer: one TILE slice per wavefront, contiguous,
// so a group of NW tiles has one row-ordered array of NW * TILE slots.
template <class AT, int NW>
__device__ __forceinline__ AT* prod_lds() {
    __shared__ AT prod[NW * TILE];
    return prod;
}

// Wavefront per tile over tiles [tb, te) (tile indices and the tables stay
// those of the whole matrix); each wavefront walks its own tiles.
// slotbits = PACK_SLOTBITS for tile-sorted storage, 0 for row order.
template <class VT, class AT, int NW, bool CACHED, bool OFF32, class Pre, class Row, class Piece, class Fin>
__device__ __forceinline__ void spmv_tiles(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const VT* __restrict__ x, const VT* xs,
                                           int hn, int64_t n, int64_t nnz, int64_t n_tiles, int64_t tb,
                                           int64_t te, int slotbits, const int32_t* __restrict__ ob, uint32_t* tk,
                                           double* head, double* tail, Pre&& pre, Row&& row, Piece&& piece,
                                           Fin&& fin) {
    const int lane = threadIdx.x & 63;
    AT* pw = prod_lds<AT, NW>() + (threadIdx.x >> 6) * TILE;
    const TileRange tr = wave_tiles<NW>(tb, te);
    const int64_t items = nnz + n;
    int64_t r_lo = 0, r_hi = 0;
    if (tr.first < tr.end) {
        r_lo = ob[tr.first];
        r_hi = ob[tr.first + 1];
    }
    for (int64_t t = tr.first; t < tr.end; t += tr.stride) {
        // Row bounds of the next tile, loaded while this one works.
        const int64_t tn = t + tr.stride;
        int64_t n_lo = 0, n_hi = 0;
        if (tn < tr.end) {
            n_lo = ob[tn];
            n_hi = ob[tn + 1];
        }
        const TileRows q = tile_rows(rp, t, r_lo, r_hi, n, items, lane, pre);
        tile_products<VT, AT, CACHED, OFF32>(col, val, x, xs, hn, q.t0, q.cnt, slotbits, pw, lane);
        wave_sync();
        tile_sums(q, pw, rp, n, n_tiles, tk, head, tail, lane, pre, row, piece, fin);
        wave_sync();
        r_lo = n_lo;
        r_hi = n_hi;
    }
}

// Group-sorted storage: the entries of each group of GROUP_TILES consecutive
// tiles are stored in column order with GROUP_SLOTBITS-bit slots (positions
// in the group's row order).  A workgroup takes NW / GROUP_TILES groups at a
// time; wavefront w loads the (w % GROUP_TILES)-th TILE of its group's stored
// entries, so one wavefront instruction gathers from a narrow column range.
// The products land in the group's row-ordered slice of the workgroup buffer,
// and after a barrier each wavefront sums its own tile.  Group sets are split
// contiguously over the eight XCDs.  Every wavefront runs the same number of
// iterations (the barriers need it).
template <class VT, class AT, int NW, bool CACHED, bool OFF32, class Pre, class Row, class Piece, class Fin>
__device__ __forceinline__ void spmv_groups(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const VT* __restrict__ val, const VT* __restrict__ x, const VT* xs,
                                            int hn, int64_t n, int64_t nnz, int64_t n_tiles,
                                            const int32_t* __restrict__ ob, uint32_t* tk, double* head,
                                            double* tail, Pre&& pre, Row&& row, Piece&& piece, Fin&& fin) {
    static_assert(NW % GROUP_TILES == 0, "whole groups per workgroup");
    constexpr int GPW = NW / GROUP_TILES;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wi = w % GROUP_TILES;
    AT* pg = prod_lds<AT, NW>() + (w / GROUP_TILES) * (GROUP_TILES * TILE);
    const int64_t items = nnz + n;
    const int64_t n_groups = (n_tiles + GROUP_TILES - 1) / GROUP_TILES;
    const int64_t n_sets = (n_groups + GPW - 1) / GPW;
    const int64_t xcd = blockIdx.x & 7, nb8 = gridDim.x >> 3;
    const int64_t lo = n_sets * xcd / 8, hi = n_sets * (xcd + 1) / 8;
    for (int64_t gs = lo + (blockIdx.x >> 3); gs < hi; gs += nb8) {
        const int64_t tg = (gs * GPW + w / GROUP_TILES) * GROUP_TILES;
        const bool live = tg < n_tiles;
        const int64_t te = min<int64_t>(tg + GROUP_TILES, n_tiles);
        const int64_t g0 = live ? tg * TILE - ob[tg] : nnz;
        const int64_t gend = !live || te >= n_tiles ? nnz : te * TILE - ob[te];
        const int64_t t = tg + wi;
        const bool has = t < n_tiles;
        TileRows q{};
        if (has) q = tile_rows(rp, t, ob[t], ob[t + 1], n, items, lane, pre);
        const int cw = (int)max<int64_t>(0, min<int64_t>(TILE, gend - g0 - (int64_t)wi * TILE));
        tile_products<VT, AT, CACHED, OFF32>(col, val, x, xs, hn, g0 + (int64_t)wi * TILE, cw, GROUP_SLOTBITS, pg,
                                              lane);
        __syncthreads();
        if (has) tile_sums(q, pg + (q.t0 - g0), rp, n, n_tiles, tk, head, tail, lane, pre, row, piece, fin);
        __syncthreads();
    }
}

// ------------------------------------------------------------ sweep blocks
// The sweep-block copy of the relabelled matrix (layout in lz_internal.h).
struct SweepArgs {
    const int32_t* ob;    // first owned row of every block (nb + 1)
    const int64_t* e;     // first entry of every block (nb + 1)
    const int32_t* col;   // columns, column order within each block
    const uint16_t* rl;   // row of each entry relative to ob[b]
    const void* val;
    int64_t nb;
};
// Entries per lane in flight.  R-MAT 26 step SpMV with 8 / 12 / 16: FP64
// 14.32 / 13.77 / 13.78 ms, FP32 12.49 / 12.40 / 12.45, BF16 9.66 / 9.58 /
// 9.67 (the LDS of the row sums already limits occupancy to two wavefronts
// per SIMD, so the extra registers cost nothing).
constexpr int SW_U = 12;
// Rows per block, wavefronts per workgroup (their row sums fill the LDS, so
// one workgroup per CU) and grid, per storage precision.  Measured on
// MI355X, R-MAT scale 26 step SpMV (rows/wavefronts/grid): FP64 4096/4/1024
// 14.3 ms, 4096/4/512 15.0, 2048/8/512 16.5; FP32 2048/8/512 12.4 ms,
// 4096/4/1024 12.6, 4096/4/512 13.0, 2048/4/512 13.2; BF16 2048/8/512
// 9.7 ms, 2048/4/512 10.3, 4096/4/1024 11.7, 4096/4/512 12.3.
template <int P> struct SweepShape { static constexpr int ROWS = 2048, WAVES = 8, GRID = 512; };
template <> struct SweepShape<0> { static constexpr int ROWS = 4096, WAVES = 4, GRID = 1024; };
static_assert(SweepShape<0>::ROWS == sweep_rows(0) && SweepShape<1>::ROWS == sweep_rows(1) &&
                  SweepShape<2>::ROWS == sweep_rows(2) && SweepShape<0>::ROWS <= SW_ROWS_MAX,
              "sweep block rows");

// Wavefront per sweep block, blocks dealt round-robin over all wavefronts
// of the grid.  A block zeroes its row sums in LDS (owned rows, then the row
// continuing past it), walks its entries in stored (column) order, 64 * SW_U
// at a time, adding each product into its row's sum with an LDS atomic, and
// then hands every owned row to the epilogue, one lane per row.  The sums
// are binary64 in every storage mode: a hub row can put all of a block's
// 2^18 products into one sum, and a binary32 chain that long loses about
// sqrt(2^18) units of its last place (on a matrix with such rows, binary32
// sums put the FP32-storage Ritz values 1.6e-6 from the FP64 ones); the
// products of FP32 and BF16 values are exact in binary64.  Split rows
// work as for tiles: the block that owns a row whose entries began in
// earlier blocks publishes a head piece, every block a row continues past
// publishes a tail piece, and the last piece to arrive on the owner's ticket
// adds them in block order.  Each wavefront has its own sums and adds into
// them in a fixed instruction order, so the result does not depend on timing.
template <class VT, int NW, int ROWS, class Pre, class Row, class Piece, class Fin>
__device__ __forceinline__ void spmv_sweep(const SweepArgs& sw, const int64_t* __restrict__ rp,
                                           const VT* __restrict__ x, int64_t n, uint32_t* tk, double* head,
                                           double* tail, Pre&& pre, Row&& row, Piece&& piece, Fin&& fin) {
    constexpr int64_t ITEMS = (int64_t)SW_W * ROWS;
    __shared__ double ys_all[NW][ROWS + 1];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double* ys = ys_all[w];
    const int32_t* __restrict__ col = sw.col;
    const uint16_t* __restrict__ rlv = sw.rl;
    const VT* __restrict__ val = (const VT*)sw.val;
    const int64_t nw = (int64_t)gridDim.x * NW;
    for (int64_t b = (int64_t)blockIdx.x * NW + w; b < sw.nb; b += nw) {
        const int64_t r0 = sw.ob[b], r1 = sw.ob[b + 1];
        const int64_t e0 = sw.e[b], e1 = sw.e[b + 1];
        const int nown = (int)(r1 - r0);
        for (int i = lane; i <= nown; i += 64) ys[i] = 0.0;
        wave_sync();
        for (int64_t base = e0; base < e1; base += 64 * SW_U) {
            int c[SW_U], r[SW_U];
            VT v[SW_U];
#pragma unroll
            for (int q = 0; q < SW_U; ++q) {
                const int64_t k = min(base + q * 64 + lane, e1 - 1);
                c[q] = __builtin_nontemporal_load(col + k);
                r[q] = (int)__builtin_nontemporal_load(rlv + k);
                v[q] = __builtin_nontemporal_load(val + k);
            }
#pragma unroll
            for (int q = 0; q < SW_U; ++q) {
                const bool warm = (uint32_t)c[q] < GATHER_WARM_BYTES / (uint32_t)sizeof(VT);
                const VT xv = warm ? x[c[q]] : __builtin_nontemporal_load(x + c[q]);
                if (base + q * 64 + lane < e1)
                    __hip_atomic_fetch_add(ys + min(r[q], nown), to_a(v[q], 0.0) * to_a(xv, 0.0),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
        wave_sync();
        const bool split_head = nown > 0 && rp[r0] < e0;
        double head_s = 0.0;
        for (int i = lane; i < nown; i += 64) {
            const int64_t rr = r0 + i;
            const double s = ys[i];
            if (i == 0 && split_head) {
                head_s = s;
                piece(rr, s);
            } else {
                row(rr, s, pre(rr));
            }
        }
        if (split_head) {
            if (lane == 0) st_dev(&head[b], head_s);
            const int64_t t1 = (rp[r0] + SW_W * r0) / ITEMS;
            if (last_wave(&tk[b], (uint32_t)(b - t1 + 1))) {
                const double tot = split_total(head, tail, t1, b, lane);
                if (lane == 0) fin(r0, tot);
            }
        }
        if (r1 < n) {
            const int64_t rb = rp[r1];
            if (rb < e1) {
                const double s = ys[nown];
                if (lane == 0) {
                    piece(r1, s);
                    st_dev(&tail[b], s);
                }
                const int64_t t1 = (rb + SW_W * r1) / ITEMS, t2 = (rp[r1 + 1] + SW_W * r1) / ITEMS;
                if (last_wave(&tk[t2], (uint32_t)(t2 - t1 + 1))) {
                    const double tot = split_total(head, tail, t1, t2, lane);
                    if (lane == 0) fin(r1, tot);
                }
            }
        }
        wave_sync();
    }
}

}  // namespace lz
