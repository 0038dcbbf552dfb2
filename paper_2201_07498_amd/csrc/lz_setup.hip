// Per-matrix setup of a solve on gfx950: input checks, the optional
// hub-first relabelling of the matrix and the SpMV tile table.
//
// Hub-first relabelling.  Algorithm 1 runs unchanged on P A P^T for a
// permutation P; its Ritz values are those of A and its Ritz vectors are
// P y.  On power-law graphs most gathers of x hit a few high-degree
// vertices, and listing those vertices first packs the hot part of x into
// few cache lines (it stays in L1/L2 instead of crossing the fabric).  The
// permutation is a stable counting sort of the rows by degree class
// (half-octaves of degree + 1, largest first), so rows of one class keep
// their original order.  Everything random the method draws (start and
// restart vectors) is drawn by original row index, and the Ritz vectors are
// written back in original order, so the Krylov sequence is the one of the
// original problem up to rounding.
//
// The decision is taken on the device (the caller's stream never waits for
// the host): with LZ_REORDER_AUTO the matrix is relabelled when it is large
// and skewed (n >= REORDER_MIN_N and the longest row at least REORDER_SKEW
// times the mean row length).
#include <algorithm>

#include "../../include/lanczos_topk.h"
#include "lz_spmv.h"

namespace lz {

constexpr int64_t REORDER_MIN_N = 1 << 17;
constexpr double REORDER_SKEW = 32.0;
constexpr int CHR = 4096;          // rows per counting-sort chunk (one workgroup)
constexpr int NKEY = 64;           // degree classes

__global__ void k_reset(State* st, int m, int K, int reorth, int reorder, double u_s, double u_w, uint64_t seed,
                        int arith) {
    uint64_t* p = reinterpret_cast<uint64_t*>(st);
    const size_t words = sizeof(State) / 8;
    for (size_t i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->m = m;
        st->K = K;
        st->reorth = reorth;
        st->reorder = reorder;
        st->u_s = u_s;
        st->u_w = u_w;
        st->seed = seed;
        st->arith = arith;
    }
}

// Input checks before any kernel indexes memory through the CSR arrays:
// rowptr[0] = 0, rowptr[n] = nnz, rows non-decreasing, 0 <= col < n.  Also
// finds the longest row.  With col null (entries in host memory) only the
// row pointers are checked here; k_validate_cols checks each slab.
__global__ __launch_bounds__(BLOCK) void k_validate(State* st, const int64_t* rp, const int32_t* col, int64_t n,
                                                    int64_t nnz) {
    bool bad = false;
    uint64_t mx = 0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t0 == 0) bad |= (rp[0] != 0) || (rp[n] != nnz);
    for (int64_t r = t0; r < n; r += stride) {
        const int64_t d = rp[r + 1] - rp[r];
        bad |= d < 0;
        mx = d > 0 && (uint64_t)d > mx ? (uint64_t)d : mx;
    }
    if (col)
        for (int64_t p = t0; p < nnz; p += stride) bad |= (col[p] < 0) || ((int64_t)col[p] >= n);
    if (bad) __hip_atomic_store(&st->status, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // One atomic per workgroup (the grid is capped, so contention is small).
    __shared__ uint64_t smx[BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t v = __shfl_xor(mx, o, 64);
        mx = v > mx ? v : mx;
    }
    if ((threadIdx.x & 63) == 0) smx[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < BLOCK / 64; ++i) mx = smx[i] > mx ? smx[i] : mx;
        if (mx > 0)
            __hip_atomic_fetch_max(&st->maxdeg, (unsigned long long)mx, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Column checks of the entries [e0, e1) of a slab (col indexed by matrix
// entry), before any kernel gathers through them.
__global__ __launch_bounds__(BLOCK) void k_validate_cols(State* st, const int32_t* col, int64_t e0, int64_t e1,
                                                         int64_t n) {
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t p = e0 + (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < e1; p += stride)
        bad |= (col[p] < 0) || ((int64_t)col[p] >= n);
    if (bad) __hip_atomic_store(&st->status, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

void launch_validate_cols(State* st, const int32_t* col, int64_t e0, int64_t e1, int64_t n, hipStream_t s) {
    if (e1 <= e0) return;
    const int g = (int)std::min<int64_t>((e1 - e0 + BLOCK - 1) / BLOCK, 1024);
    hipLaunchKernelGGL(k_validate_cols, dim3(g), dim3(BLOCK), 0, s, st, col, e0, e1, n);
}

// Chooses the matrix of the solve and publishes its pointers in the state.
__global__ void k_reorder_decide(State* st, const int64_t* rp, const int32_t* col, const void* val, int64_t n,
                                 int64_t nnz, int64_t* rp2, int32_t* col2, void* val2, int32_t* perm,
                                 int32_t* iperm, int sweep) {
    if (threadIdx.x != 0) return;
    const int opt = st->reorder;
    bool use = false;
    if (st->status == 0 && n > 1 && nnz > 0) {
        if (opt == LZ_REORDER_HUBS) use = true;
        if (opt == LZ_REORDER_AUTO)
            use = n >= REORDER_MIN_N && (double)st->maxdeg * (double)n >= REORDER_SKEW * (double)nnz;
    }
    st->reordered = use ? 1 : 0;
    st->packed = !use ? PACK_NONE
                 : sweep ? PACK_SWEEP
                 : n <= (int64_t(1) << GROUP_COLBITS) ? PACK_GROUP
                 : n < (int64_t(1) << PACK_COLBITS) ? PACK_TILE : PACK_NONE;
    st->crp = use ? rp2 : rp;
    st->ccol = use ? col2 : col;
    st->cval = use ? val2 : val;
    st->perm = use ? perm : nullptr;
    st->iperm = use ? iperm : nullptr;
}

// ------------------------------------------------------------- scans
constexpr int SCAN_PER = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_PER;

__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* sh, uint64_t* total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < BLOCK; o <<= 1) {
        const uint64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t incl = sh[threadIdx.x];
    *total = sh[BLOCK - 1];
    __syncthreads();
    return incl - v;
}

// Exclusive scan of x[0..n) in place, in three kernels; skipped unless
// *gate is set.
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const int32_t* gate, const uint64_t* x, int64_t n,
                                                       uint64_t* bsum) {
    __shared__ uint64_t sh[BLOCK];
    if (!*gate) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
    for (int i = 0; i < SCAN_PER; ++i) {
        const int64_t r = base + (int64_t)threadIdx.x * SCAN_PER + i;
        if (r < n) s += x[r];
    }
    uint64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BLOCK) void k_scan_top(const int32_t* gate, uint64_t* bsum, int64_t nb) {
    __shared__ uint64_t sh[BLOCK];
    if (!*gate) return;
    const int64_t per = (nb + BLOCK - 1) / BLOCK;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    uint64_t s = 0;
    for (int64_t i = 0; i < per; ++i)
        if (b0 + i < nb) s += bsum[b0 + i];
    uint64_t tot;
    uint64_t run = block_exclusive_scan(s, sh, &tot);
    for (int64_t i = 0; i < per; ++i)
        if (b0 + i < nb) {
            const uint64_t v = bsum[b0 + i];
            bsum[b0 + i] = run;
            run += v;
        }
    if (threadIdx.x == 0) bsum[nb] = tot;
}

__global__ __launch_bounds__(BLOCK) void k_scan_apply(const int32_t* gate, uint64_t* x, int64_t n,
                                                      const uint64_t* bsum) {
    __shared__ uint64_t sh[BLOCK];
    if (!*gate) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    uint64_t v[SCAN_PER];
    uint64_t s = 0;
    for (int i = 0; i < SCAN_PER; ++i) {
        v[i] = (base + i < n) ? x[base + i] : 0ull;
        s += v[i];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_scan(s, sh, &tot) + bsum[blockIdx.x];
    for (int i = 0; i < SCAN_PER; ++i)
        if (base + i < n) {
            x[base + i] = run;
            run += v[i];
        }
}

static void scan(const int32_t* gate, uint64_t* x, int64_t n, uint64_t* bsum, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(BLOCK), 0, s, gate, x, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, s, gate, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(BLOCK), 0, s, gate, x, n, bsum);
}

// ------------------------------------------------------- relabelling
// Degree class: 63 - floor(log2((d+1)^2)), so longer rows sort first.
__device__ __forceinline__ int degree_key(int64_t d) {
    uint64_t x = (uint64_t)min<int64_t>(d, (int64_t(1) << 31) - 1) + 1u;
    x *= x;
    return __builtin_clzll(x);       // = 63 - floor(log2 x), in [2, 63]
}

// hist[key * nch + c] = rows of class key in chunk c.
__global__ __launch_bounds__(BLOCK) void k_rl_hist(const State* st, const int64_t* rp, int64_t n, int64_t nch,
                                                   uint64_t* hist) {
    __shared__ uint32_t cnt[NKEY];
    if (!st->reordered) return;
    const int64_t c = blockIdx.x;
    if (threadIdx.x < NKEY) cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < CHR; i += BLOCK) {
        const int64_t r = c * CHR + i;
        if (r < n) atomicAdd(&cnt[degree_key(rp[r + 1] - rp[r])], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NKEY) hist[(int64_t)threadIdx.x * nch + c] = cnt[threadIdx.x];
}

// Stable ranks: new position = (rows of earlier classes) + (rows of this
// class in earlier chunks) + (rows of this class earlier in this chunk).
__global__ __launch_bounds__(BLOCK) void k_rl_rank(const State* st, const int64_t* rp, int64_t n, int64_t nch,
                                                   const uint64_t* off, int32_t* perm, int32_t* iperm) {
    __shared__ uint64_t run[NKEY];
    __shared__ uint32_t wcnt[WAVES][NKEY];
    if (!st->reordered) return;
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < NKEY) run[threadIdx.x] = off[(int64_t)threadIdx.x * nch + c];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int base = 0; base < CHR; base += BLOCK) {
        for (int i = threadIdx.x; i < WAVES * NKEY; i += BLOCK) wcnt[i / NKEY][i % NKEY] = 0u;
        __syncthreads();
        const int64_t r = c * CHR + base + threadIdx.x;
        const bool valid = r < n;
        const int key = valid ? degree_key(rp[r + 1] - rp[r]) : 0;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 6; ++bit) {
            const bool on = (key >> bit) & 1;
            const uint64_t bb = __ballot(valid && on);
            same &= on ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (valid && rank == 0) wcnt[w][key] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint64_t pos = run[key] + rank;
            for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][key];
            perm[pos] = (int32_t)r;
            iperm[r] = (int32_t)pos;
        }
        __syncthreads();
        if (threadIdx.x < NKEY) {
            uint64_t add = 0;
            for (int ww = 0; ww < WAVES; ++ww) add += wcnt[ww][threadIdx.x];
            run[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

// Row lengths of the relabelled matrix into rp2 (scanned afterwards).
__global__ __launch_bounds__(BLOCK) void k_rl_rowlen(const State* st, const int64_t* rp, int64_t n,
                                                     const int32_t* perm, int64_t* rp2, int64_t nnz) {
    if (!st->reordered) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t r = perm[i];
        rp2[i] = rp[r + 1] - rp[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) rp2[n] = nnz;
}

// Copies every row to its new place, columns relabelled.  One wavefront per
// SpMV tile of the relabelled matrix (balanced over entries and rows).  The
// tile's rows are staged in LDS once: their first new position rp2 and the
// shift from new to old position (rp[perm[row]] - rp2[row]).  Each lane then
// takes its 16 entries together: a fixed-step search over the staged rows,
// then all 16 col/val loads, then all 16 iperm gathers, so a tile costs two
// rounds of requests.  For n < 2^22 the tile is then sorted by column in
// LDS and stored packed (col << 10 | position in row order): the SpMV's
// gathers of one wavefront instruction then hit neighbouring columns.
constexpr int FILL_WAVES = 2;

// Bitonic sort, ascending, of the N keys of the threads 0 .. N/16-1 of a
// workgroup: element tid*16 + r is kr[r] of thread tid.  Exchanges between
// elements less than 16 apart stay in a thread's registers, those within a
// wavefront are lane shuffles, and those between wavefronts (N > 1024) go
// through xbuf (N keys of LDS) between barriers, so every thread of the
// workgroup must call it.
template <int N>
__device__ __forceinline__ void sort_keys(uint32_t (&kr)[TP], int tid, uint32_t* xbuf) {
#pragma unroll
    for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64 * TP) {
#pragma unroll
                for (int r = 0; r < TP; ++r) xbuf[tid * TP + r] = kr[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < TP; ++r) {
                    const int i = tid * TP + r;
                    const uint32_t o = xbuf[i ^ j];
                    const uint32_t lo = min(kr[r], o), hi = max(kr[r], o);
                    kr[r] = (((i & j) == 0) == ((i & kk) == 0)) ? lo : hi;
                }
                __syncthreads();
            } else if (j >= TP) {
#pragma unroll
                for (int r = 0; r < TP; ++r) {
                    const int i = tid * TP + r;
                    const uint32_t o = (uint32_t)__shfl_xor((int)kr[r], j / TP, 64);
                    const uint32_t lo = min(kr[r], o), hi = max(kr[r], o);
                    kr[r] = (((i & j) == 0) == ((i & kk) == 0)) ? lo : hi;
                }
            } else {
#pragma unroll
                for (int r = 0; r < TP; ++r) {
                    if ((r & j) != 0) continue;
                    const int r2 = r | j;
                    const bool asc = ((tid * TP + r) & kk) == 0;
                    const uint32_t a = kr[r], b = kr[r2];
                    const bool sw = (a > b) == asc;
                    kr[r] = sw ? b : a;
                    kr[r2] = sw ? a : b;
                }
            }
        }
    }
}

// One wavefront's share of the fill: the 16 entries of each lane of tile t
// (entry t0 + e*64 + lane, clamped to the tile) with columns relabelled.  The
// tile's rows are staged in s/d first: their first new position relative to
// the tile (clamped at -1: only the first row can start before it) and the
// shift from new to old position (rp[perm[row]] - rp2[row]).  Returns the
// tile's entry count (0: row ends only, nothing loaded).
template <class VT>
__device__ __forceinline__ int fill_tile_gather(int64_t t, const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                int64_t n, int64_t nnz, const int32_t* __restrict__ ob,
                                                const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                                                const int64_t* __restrict__ rp2, int32_t* s, int64_t* d, int lane,
                                                int64_t* t0_out, int32_t (&c)[TP], VT (&v)[TP],
                                                int32_t (&rows)[TP]) {
    const int64_t r_lo = ob[t], r_hi = ob[t + 1];
    const int64_t t0 = t * TILE - r_lo;
    *t0_out = t0;
    const int cnt = (int)(min<int64_t>((t + 1) * TILE, nnz + n) - r_hi - t0);
    if (cnt <= 0) return 0;
    // Rows r_lo .. r_last touch the tile (at most TILE + 1 of them).
    const int64_t r_last = min(r_hi, n - 1);
    const int nr = (int)(r_last - r_lo + 1);
    for (int i = lane; i <= nr; i += 64) s[i] = (int32_t)max<int64_t>(rp2[r_lo + i] - t0, -1);
    for (int i = lane; i < nr; i += 64) d[i] = rp[perm[r_lo + i]] - rp2[r_lo + i];
    wave_sync();
    int64_t src[TP];
#pragma unroll
    for (int e = 0; e < TP; ++e) {
        const int k = min(e * 64 + lane, cnt - 1);
        // Largest i < nr with s[i] <= k (the row whose range holds entry t0 + k).
        int lo = 0;
#pragma unroll
        for (int step = TILE; step > 0; step >>= 1)
            if (lo + step < nr && s[lo + step] <= k) lo += step;
        src[e] = t0 + k + d[lo];
        rows[e] = (int32_t)(r_lo + lo);
    }
#pragma unroll
    for (int e = 0; e < TP; ++e) {
        c[e] = col[src[e]];
        v[e] = val[src[e]];
    }
#pragma unroll
    for (int e = 0; e < TP; ++e) c[e] = iperm[c[e]];
    return cnt;
}

template <class VT>
__global__ __launch_bounds__(FILL_WAVES * 64) void k_rl_fill(const State* st, const int64_t* __restrict__ rp,
                                                            const int32_t* __restrict__ col,
                                                            const VT* __restrict__ val, int64_t n, int64_t nnz,
                                                            int64_t n_tiles, const int32_t* __restrict__ ob,
                                                            const int32_t* __restrict__ perm,
                                                            const int32_t* __restrict__ iperm,
                                                            const int64_t* __restrict__ rp2,
                                                            int32_t* __restrict__ col2, VT* __restrict__ val2,
                                                            const int32_t* __restrict__ swob,
                                                            const int64_t* __restrict__ swe, int64_t sw_items,
                                                            uint32_t* __restrict__ swvin) {
    __shared__ int32_t srp[FILL_WAVES][TILE + 2];
    __shared__ int64_t sdel[FILL_WAVES][TILE + 1];
    if (!st->reordered) return;
    if (st->packed == PACK_GROUP) return;     // k_rl_fill_group builds it
    const bool packed = st->packed == PACK_TILE;
    const bool sweep = st->packed == PACK_SWEEP && swvin != nullptr;
    const int lane = threadIdx.x & 63;
    int32_t* s = srp[threadIdx.x >> 6];
    int64_t* d = sdel[threadIdx.x >> 6];
    const TileRange tr = wave_tiles<FILL_WAVES>(0, n_tiles);
    for (int64_t t = tr.first; t < tr.end; t += tr.stride) {
        int32_t c[TP];
        VT v[TP];
        int32_t rows[TP];
        int64_t t0 = 0;
        const int cnt = fill_tile_gather(t, rp, col, val, n, nnz, ob, perm, iperm, rp2, s, d, lane, &t0, c, v, rows);
        if (cnt <= 0) continue;                   // row ends only: no entries to move
        if (!packed) {
#pragma unroll
            for (int e = 0; e < TP; ++e) {
                const int k = e * 64 + lane;
                if (k < cnt) {
                    col2[t0 + k] = c[e];
                    val2[t0 + k] = v[e];
                }
            }
            if (sweep) {
                // Sort payload of the sweep blocks: the entry's row within its
                // block (high bits) and its position in the block.
#pragma unroll
                for (int e = 0; e < TP; ++e) {
                    const int k = e * 64 + lane;
                    if (k < cnt) {
                        const int64_t pos = t0 + k, r = rows[e];
                        const int64_t b = (pos + SW_W * r) / sw_items;
                        swvin[pos] = ((uint32_t)(r - swob[b]) << SW_POSBITS) | (uint32_t)(pos - swe[b]);
                    }
                }
            }
            wave_sync();
            continue;
        }
        // Column-sorted tile: keys (col << 10 | position) go through the LDS
        // of the row search (no longer read) so that each lane holds 16
        // consecutive ones, the wavefront sorts them in registers (unique
        // keys, so the order is fixed; padding sorts last), and the sorted
        // keys come back through LDS for coalesced stores with their values.
        wave_sync();
        uint32_t* key = reinterpret_cast<uint32_t*>(s);
        VT* sv = reinterpret_cast<VT*>(d);
#pragma unroll
        for (int e = 0; e < TP; ++e) {
            const int k = e * 64 + lane;
            key[k] = k < cnt ? ((uint32_t)c[e] << PACK_SLOTBITS) | (uint32_t)k : 0xffffffffu;
            sv[k] = v[e];
        }
        wave_sync();
        uint32_t kr[TP];
#pragma unroll
        for (int r = 0; r < TP; ++r) kr[r] = key[lane * TP + r];
        sort_keys<TILE>(kr, lane, nullptr);
        wave_sync();
#pragma unroll
        for (int r = 0; r < TP; ++r) key[lane * TP + r] = kr[r];
        wave_sync();
#pragma unroll
        for (int e = 0; e < TP; ++e) {
            const int k = e * 64 + lane;
            if (k < cnt) {
                const uint32_t kv = key[k];
                col2[t0 + k] = (int32_t)kv;
                val2[t0 + k] = sv[kv & PACK_SLOTMASK];
            }
        }
        wave_sync();
    }
}

// Group-sorted fill (n <= 2^20): a workgroup of GROUP_TILES wavefronts
// takes a group of consecutive tiles; each wavefront gathers its tile as
// above, the keys (col << 12 | position in the group) and values go to LDS
// by position, the workgroup sorts the keys, and the sorted keys are stored
// with their values.
template <class VT>
__global__ __launch_bounds__(BLOCK) void k_rl_fill_group(const State* st, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                         int64_t n, int64_t nnz, int64_t n_tiles,
                                                         const int32_t* __restrict__ ob,
                                                         const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ iperm,
                                                         const int64_t* __restrict__ rp2, int32_t* __restrict__ col2,
                                                         VT* __restrict__ val2) {
    static_assert(BLOCK / 64 == GROUP_TILES, "one wavefront per tile of a group");
    constexpr int GN = GROUP_TILES * TILE;
    __shared__ int32_t srp[GROUP_TILES][TILE + 2];
    __shared__ int64_t sdel[GROUP_TILES][TILE + 1];
    static_assert(sizeof(srp) >= GN * sizeof(uint32_t) && sizeof(sdel) >= GN * sizeof(VT), "LDS reuse");
    if (!st->reordered || st->packed != PACK_GROUP) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int32_t* s = srp[w];
    int64_t* d = sdel[w];
    uint32_t* key = reinterpret_cast<uint32_t*>(&srp[0][0]);
    VT* sv = reinterpret_cast<VT*>(&sdel[0][0]);
    const int64_t n_groups = (n_tiles + GROUP_TILES - 1) / GROUP_TILES;
    const int64_t xcd = blockIdx.x & 7, nb8 = gridDim.x >> 3;
    const int64_t lo = n_groups * xcd / 8, hi = n_groups * (xcd + 1) / 8;
    for (int64_t g = lo + (blockIdx.x >> 3); g < hi; g += nb8) {
        const int64_t tg = g * GROUP_TILES, te = min<int64_t>(tg + GROUP_TILES, n_tiles);
        const int64_t g0 = tg * TILE - ob[tg];
        const int64_t gend = te >= n_tiles ? nnz : te * TILE - ob[te];
        const int ne = (int)(gend - g0);
        const int64_t t = tg + w;
        int32_t c[TP];
        VT v[TP];
        int64_t t0 = 0;
        int32_t rows[TP];
        const int cnt = t < n_tiles ? fill_tile_gather(t, rp, col, val, n, nnz, ob, perm, iperm, rp2, s, d, lane,
                                                       &t0, c, v, rows)
                                    : 0;
        __syncthreads();                          // the key and value arrays overlap every wavefront's s, d
        const int off = (int)(t0 - g0);
#pragma unroll
        for (int e = 0; e < TP; ++e) {
            const int k = e * 64 + lane;
            if (k < cnt) {
                key[off + k] = ((uint32_t)c[e] << GROUP_SLOTBITS) | (uint32_t)(off + k);
                sv[off + k] = v[e];
            }
        }
        for (int p = ne + tid; p < GN; p += BLOCK) key[p] = 0xffffffffu;
        __syncthreads();
        uint32_t kr[TP];
#pragma unroll
        for (int r = 0; r < TP; ++r) kr[r] = key[tid * TP + r];
        __syncthreads();
        sort_keys<GN>(kr, tid, key);
#pragma unroll
        for (int r = 0; r < TP; ++r) key[tid * TP + r] = kr[r];
        __syncthreads();
        for (int p = tid; p < ne; p += BLOCK) {
            const uint32_t kv = key[p];
            col2[g0 + p] = (int32_t)kv;
            val2[g0 + p] = sv[kv & GROUP_SLOTMASK];
        }
        __syncthreads();
    }
}

// Tile table over the solve's matrix: ob[t] = first row owned by tile t,
// ob[n_tiles] = n; clears the split-row tickets.  Owners are non-decreasing
// in r, so row r writes the entries of the tiles after its predecessor's
// owner up to its own.
__global__ __launch_bounds__(BLOCK) void k_setup_tiles(const State* st, int64_t n, int64_t n_tiles, int32_t* ob,
                                                       uint32_t* tk) {
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    for (int64_t t = t0; t < n_tiles; t += stride) tk[t] = 0u;
    if (t0 == 0) ob[n_tiles] = (int32_t)n;
    if (st->status != 0) return;
    const int64_t* rp = st->crp;
    for (int64_t r = t0; r < n; r += stride) {
        const int64_t own = row_owner(rp, r, n_tiles);
        const int64_t prev = r > 0 ? row_owner(rp, r - 1, n_tiles) : -1;
        for (int64_t t = prev + 1; t <= own; ++t) ob[t] = (int32_t)r;
    }
}

bool host_relabel_decision(const int64_t* rp, int64_t n, int64_t nnz, int reorder) {
    if (n <= 1 || nnz <= 0 || reorder == LZ_REORDER_OFF) return false;
    if (reorder == LZ_REORDER_HUBS) return true;
    if (n < REORDER_MIN_N) return false;
    int64_t mx = 0;
    for (int64_t r = 0; r < n; ++r) mx = std::max<int64_t>(mx, rp[r + 1] - rp[r]);
    return (double)mx * (double)n >= REORDER_SKEW * (double)nnz;
}

hipError_t launch_setup(const Plan& p, const Bufs& b, const Csr& a, uint64_t seed, int reorth, int reorder,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(BLOCK), 0, s, b.st, p.m, p.K, reorth, reorder, unit_roundoff(p.prec),
                       work_roundoff(p.prec), seed, p.fff);
    const int64_t n = a.n, nnz = a.nnz;
    const int g = (int)std::min<int64_t>((n + BLOCK - 1) / BLOCK, 8192);
    const int gv = (int)std::min<int64_t>((std::max(n, nnz) + BLOCK - 1) / BLOCK, 1024);
    hipLaunchKernelGGL(k_validate, dim3(gv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col, n, nnz);
    hipLaunchKernelGGL(k_reorder_decide, dim3(1), dim3(64), 0, s, b.st, a.rowptr, a.col, a.val, n, nnz, b.rp2,
                       b.col2, b.val2, b.perm, b.iperm, p.sweep);
    const int32_t* gate = &b.st->reordered;
    if (reorder != LZ_REORDER_OFF) {
        const int64_t nch = (n + CHR - 1) / CHR;
        hipLaunchKernelGGL(k_rl_hist, dim3((unsigned)nch), dim3(BLOCK), 0, s, b.st, a.rowptr, n, nch, b.scan);
        scan(gate, b.scan, NKEY * nch, b.bsum, s);
        hipLaunchKernelGGL(k_rl_rank, dim3((unsigned)nch), dim3(BLOCK), 0, s, b.st, a.rowptr, n, nch, b.scan,
                           b.perm, b.iperm);
        hipLaunchKernelGGL(k_rl_rowlen, dim3(g), dim3(BLOCK), 0, s, b.st, a.rowptr, n, b.perm, b.rp2, nnz);
        scan(gate, (uint64_t*)b.rp2, n, b.bsum, s);
    }
    hipLaunchKernelGGL(k_setup_tiles, dim3(g), dim3(BLOCK), 0, s, b.st, n, p.n_tiles, b.ob, b.tk);
    if (reorder != LZ_REORDER_OFF) {
        launch_sweep_blocks(p, b, s);             // the relabelling fill writes the sort payload by block
        switch (p.prec) {
            case 0:
                hipLaunchKernelGGL(k_rl_fill<double>, dim3(p.g_tile * (WAVES / FILL_WAVES)), dim3(FILL_WAVES * 64), 0, s, b.st, a.rowptr, a.col,
                                   (const double*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (double*)b.val2, b.swob, b.swe, p.sw_items, b.swvin);
                break;
            case 1:
                hipLaunchKernelGGL(k_rl_fill<float>, dim3(p.g_tile * (WAVES / FILL_WAVES)), dim3(FILL_WAVES * 64), 0, s, b.st, a.rowptr, a.col,
                                   (const float*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (float*)b.val2, b.swob, b.swe, p.sw_items, b.swvin);
                break;
            default:
                hipLaunchKernelGGL(k_rl_fill<uint16_t>, dim3(p.g_tile * (WAVES / FILL_WAVES)), dim3(FILL_WAVES * 64), 0, s, b.st, a.rowptr, a.col,
                                   (const uint16_t*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (uint16_t*)b.val2, b.swob, b.swe, p.sw_items, b.swvin);
                break;
        }
        // Group-sorted copy (decided on the device; the kernel returns unless
        // the state asks for it).
        const int64_t n_groups = (p.n_tiles + GROUP_TILES - 1) / GROUP_TILES;
        const int gg = (int)((std::min<int64_t>(n_groups, 4096) + 7) / 8 * 8);
        switch (p.prec) {
            case 0:
                hipLaunchKernelGGL(k_rl_fill_group<double>, dim3(gg), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                                   (const double*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (double*)b.val2);
                break;
            case 1:
                hipLaunchKernelGGL(k_rl_fill_group<float>, dim3(gg), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                                   (const float*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (float*)b.val2);
                break;
            default:
                hipLaunchKernelGGL(k_rl_fill_group<uint16_t>, dim3(gg), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                                   (const uint16_t*)a.val, n, nnz, p.n_tiles, b.ob, b.perm, b.iperm, b.rp2, b.col2,
                                   (uint16_t*)b.val2);
                break;
        }
        const hipError_t e = launch_sweep_sort(p, b, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace lz
