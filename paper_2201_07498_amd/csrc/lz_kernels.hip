// gfx950 kernels of the Top-K Lanczos solver.
//
// One Lanczos iteration (Sec. II, Algorithm 1) is four kernels:
//   k_spmv_step      w = A v_j - beta_j v_{j-1}; alpha_j = v_j . (A v_j)
//   k_orth_dot       c  = V^T w                       (first CGS pass, dots)
//   k_orth_upd_dot   w' = w - V c;  c2 = V^T w'       (update fused with second dots)
//   k_orth_upd_store v_{j+1} = w' - V c2, stored in the basis precision; beta_{j+1}
// Every global reduction is "partials per workgroup, then the last workgroup
// to finish sums them in workgroup order", so results do not depend on
// scheduling.  Scalars (alpha, beta, c, step index) stay in device memory.
//
// The basis V is column-major with leading dimension ld (a multiple of
// LDPAD); rows n..ld-1 are kept at zero so the dense kernels need no tail
// handling.  Column k is stored unnormalised; scale[k] makes it unit length.
#include "lz_internal.h"

#include <algorithm>
#include <cmath>

namespace lz {

// ------------------------------------------------------------------ types
template <int P> struct Tr;
template <> struct Tr<0> { using V = double;   using A = double; using W = double; };
template <> struct Tr<1> { using V = float;    using A = float;  using W = float; };
template <> struct Tr<2> { using V = uint16_t; using A = float;  using W = float; };

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(uint16_t b) { return (double)__uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ double to_a(double x, double) { return x; }
__device__ __forceinline__ float to_a(float x, float) { return x; }
__device__ __forceinline__ float to_a(uint16_t b, float) { return __uint_as_float((uint32_t)b << 16); }

// Round-to-nearest-even float -> bfloat16 bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
template <class V> __device__ __forceinline__ V from_d(double x);
template <> __device__ __forceinline__ double from_d<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_d<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t from_d<uint16_t>(double x) { return f32_to_bf16((float)x); }

// SplitMix64 (Steele, Lea, Flood 2014): output r (0-based) of the stream
// started at `seed`, and the uniform double in [0,1) from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t r) {
    uint64_t z = seed + (r + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t seed, uint64_t r) {
    return (double)(splitmix64(seed, r) >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------ reductions
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256 threads of a workgroup; every thread gets the result.
template <class T> __device__ __forceinline__ T block_sum(T v, T* sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// True in exactly one workgroup: the last of the grid to pass this point.
// Partials written before the call are visible to that workgroup.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t count, int* s_flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = (t == count - 1u);
    }
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return last;
}

// Sum of x[0..cnt) in a fixed order (thread-strided, then a fixed tree).
__device__ double ordered_sum(const double* x, int64_t cnt, double* sh) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += BLOCK) s += x[i];
    return block_sum(s, sh);
}

// out[k] = mul[k] * sum_b part[b*NCMAX + k] for k < nc, b < nb (fixed order).
__device__ void reduce_columns(const double* part, int nb, int nc, const double* mul,
                               double* out, double (*sh)[64]) {
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int k0 = 0; k0 < nc; k0 += 64) {
        const int k = k0 + l;
        double s = 0.0;
        if (k < nc)
            for (int b = q; b < nb; b += 4) s += part[(int64_t)b * NCMAX + k];
        sh[q][l] = s;
        __syncthreads();
        if (q == 0 && k < nc) out[k] = mul[k] * ((sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l]));
        __syncthreads();
    }
}

// ------------------------------------------------------------------ state
__global__ void k_reset(State* st, int m, int K, int reorth, double u_s, uint64_t seed) {
    uint64_t* p = reinterpret_cast<uint64_t*>(st);
    const size_t words = sizeof(State) / 8;
    for (size_t i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->m = m;
        st->K = K;
        st->reorth = reorth;
        st->u_s = u_s;
        st->seed = seed;
    }
}

// Input checks (before any kernel indexes memory through the CSR arrays):
// rowptr[0] = 0, rowptr[n] = nnz, rows non-decreasing, 0 <= col < n.
__global__ __launch_bounds__(BLOCK) void k_validate(State* st, const int64_t* rp, const int32_t* col, int64_t n,
                                                    int64_t nnz) {
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t0 == 0) bad |= (rp[0] != 0) || (rp[n] != nnz);
    for (int64_t r = t0; r < n; r += stride) bad |= rp[r + 1] < rp[r];
    for (int64_t p = t0; p < nnz; p += stride) bad |= (col[p] < 0) || ((int64_t)col[p] >= n);
    if (bad) __hip_atomic_store(&st->status, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------ matrix partition
// Rows are cut into work items: row blocks of consecutive short rows with
// at most about 2*NB non-zeros and RMAX rows, and chunks of CH non-zeros of
// every long row (more than NB non-zeros).  Row r starts a new item when it
// is the first row, a multiple of RMAX, long, after a long row, or when the
// non-zero index crosses a multiple of NB between the start of row r-1 and
// the start of row r.
__device__ __forceinline__ bool row_starts_item(const int64_t* rp, int64_t r) {
    if (r == 0 || (r % RMAX) == 0) return true;
    const int64_t b = rp[r];
    if (rp[r + 1] - b > NB) return true;
    const int64_t a = rp[r - 1];
    if (b - a > NB) return true;
    return (a / NB) != (b / NB);
}

constexpr uint64_t LOW40 = (1ull << 40) - 1ull;

__device__ __forceinline__ uint64_t item_count(const int64_t* rp, int64_t r) {
    if (!row_starts_item(rp, r)) return 0ull;
    const int64_t len = rp[r + 1] - rp[r];
    if (len > NB) return (uint64_t)((len + CH - 1) / CH) | (1ull << 40);
    return 1ull;
}

__global__ __launch_bounds__(BLOCK) void k_setup_count(const int64_t* rp, int64_t n, uint64_t* cnt) {
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLOCK)
        cnt[r] = item_count(rp, r);
}

constexpr int SCAN_PER = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_PER;

__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* sh, uint64_t* total) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < BLOCK; o <<= 1) {
        uint64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t incl = sh[threadIdx.x];
    *total = sh[BLOCK - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const uint64_t* x, int64_t n, uint64_t* bsum) {
    __shared__ uint64_t sh[BLOCK];
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

// Exclusive scan of nb block sums in place (one workgroup); bsum[nb] = total.
__global__ __launch_bounds__(BLOCK) void k_scan_top(uint64_t* bsum, int64_t nb) {
    __shared__ uint64_t sh[BLOCK];
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

__global__ __launch_bounds__(BLOCK) void k_scan_apply(uint64_t* x, int64_t n, const uint64_t* bsum) {
    __shared__ uint64_t sh[BLOCK];
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

__global__ __launch_bounds__(BLOCK) void k_setup_items(const int64_t* rp, int64_t n, const uint64_t* off,
                                                       const uint64_t* total, int64_t items_cap,
                                                       int64_t long_cap, int2* items, int32_t* lrow,
                                                       int32_t* lfirst, int32_t* lnch, uint32_t* ltk,
                                                       State* st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t t = *total;
        const int64_t ni = (int64_t)(t & LOW40), nl = (int64_t)(t >> 40);
        if (ni > items_cap || nl > long_cap) {
            st->status = -4;   // LZ_ERR_WORKSPACE_TOO_SMALL
            st->n_items = 0;
            st->n_long = 0;
        } else {
            st->n_items = (int32_t)ni;
            st->n_long = (int32_t)nl;
        }
    }
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLOCK) {
        if (!row_starts_item(rp, r)) continue;
        const uint64_t o = off[r];
        const int64_t first = (int64_t)(o & LOW40);
        const int64_t lid = (int64_t)(o >> 40);
        const int64_t len = rp[r + 1] - rp[r];
        if (len > NB) {
            const int64_t nch = (len + CH - 1) / CH;
            if (first + nch > items_cap || lid >= long_cap) continue;
            for (int64_t c = 0; c < nch; ++c) items[first + c] = make_int2((int)(-1 - lid), (int)c);
            lrow[lid] = (int32_t)r;
            lfirst[lid] = (int32_t)first;
            lnch[lid] = (int32_t)nch;
            ltk[lid] = 0u;
        } else {
            if (first >= items_cap) continue;
            int64_t e = r + 1;
            while (e < n && !row_starts_item(rp, e)) ++e;
            items[first] = make_int2((int)r, (int)e);
        }
    }
}

// ------------------------------------------------------------ start vector
// V[:,0] = u (rounded to the basis precision), u_r = U01(SplitMix64(seed, r));
// scale[0] = 1/||u||.  Also clears w (its padding rows must stay zero).
template <int P>
__global__ __launch_bounds__(BLOCK) void k_init(State* st, typename Tr<P>::V* V, typename Tr<P>::W* w,
                                                int64_t n, int64_t ld, double* part) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    __shared__ double sh[4];
    __shared__ int s_last;
    if (st->status != 0) {                 // invalid input: no Lanczos step will run
        if (blockIdx.x == 0 && threadIdx.x == 0) st->j = st->m;
        return;
    }
    const uint64_t seed = st->seed;
    double s = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK) {
        const VT v = from_d<VT>(r < n ? u01(seed, (uint64_t)r) : 0.0);
        V[r] = v;
        w[r] = (WT)0;
        const double d = to_d(v);
        s += d * d;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(&st->ticket[TK_INIT], gridDim.x, &s_last)) {
        const double tot = ordered_sum(part, gridDim.x, sh);
        if (threadIdx.x == 0) {
            st->scale[0] = 1.0 / sqrt(tot);
            st->beta[0] = 0.0;
            st->j = 0;
            st->mode = MODE_NORMAL;
        }
    }
}

// ------------------------------------------------------------------- SpMV
// Row-block item: products of the item's non-zeros are staged in LDS with
// coalesced col/val reads and gathered x, then each row is summed by a
// power-of-two group of lanes.  Long-row chunk: the workgroup sums CH
// non-zeros; the last chunk of the row to finish adds the chunk partials in
// chunk order and runs the row epilogue.
//
// Epilogue EPI_LANCZOS: y = scale_j * (A V[:,j]); w = y - beta_j v_{j-1};
//   alpha partial += v_j[r] * y.  EPI_PLAIN: y stored as is.
enum { EPI_LANCZOS = 0, EPI_PLAIN = 1 };

template <int P, int EPI>
__global__ __launch_bounds__(BLOCK) void k_spmv(State* st, const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col,
                                                const typename Tr<P>::V* __restrict__ val,
                                                const typename Tr<P>::V* __restrict__ Vb,
                                                typename Tr<P>::W* __restrict__ w, int64_t n, int64_t ld,
                                                const int2* __restrict__ items, const int32_t* lrow,
                                                const int32_t* lfirst, const int32_t* lnch, uint32_t* ltk,
                                                double* lpart, double* lval, double* part) {
    using VT = typename Tr<P>::V;
    using AT = typename Tr<P>::A;
    using WT = typename Tr<P>::W;
    __shared__ AT prod[2 * NB];
    __shared__ double shd[4];
    __shared__ AT sha[4];
    __shared__ int s_last;

    if (st->status != 0) return;
    int j = 0;
    const VT* x = Vb;
    const VT* xp = nullptr;
    double sj = 1.0, bsc = 0.0;
    if (EPI == EPI_LANCZOS) {
        j = st->j;
        if (j >= st->m) return;
        if (st->mode == MODE_RESTART) {
            // Restart: draw a fresh random vector into w; the CGS kernels that
            // follow orthogonalise it against the basis.
            const uint64_t rs = st->seed + ((uint64_t)st->restarts << 32);
            for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK)
                w[r] = (WT)(r < n ? u01(rs, (uint64_t)r) : 0.0);
            return;
        }
        x = Vb + (int64_t)j * ld;
        xp = j > 0 ? Vb + (int64_t)(j - 1) * ld : nullptr;
        sj = st->scale[j];
        bsc = j > 0 ? st->beta[j] * st->scale[j - 1] : 0.0;
    }
    const int nitems = st->n_items;
    const int tid = threadIdx.x;
    double apart = 0.0;

    auto epilogue = [&](int64_t r, double acc) {
        if (EPI == EPI_LANCZOS) {
            const double y = sj * acc;
            apart += sj * to_d(x[r]) * y;
            const double wp = xp ? bsc * to_d(xp[r]) : 0.0;
            w[r] = (WT)(y - wp);
        } else {
            w[r] = (WT)acc;
        }
    };

    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        if (item.x >= 0) {
            const int64_t rs = item.x, re = item.y;
            const int64_t ps = rp[rs];
            const int64_t cnt64 = rp[re] - ps;
            if (cnt64 < 0 || cnt64 > 2 * NB) {      // cannot happen for a validated partition
                if (tid == 0) st->status = -4;
                continue;
            }
            const int cnt = (int)cnt64;
            for (int t = tid; t < cnt; t += BLOCK)
                prod[t] = to_a(val[ps + t], AT(0)) * to_a(x[col[ps + t]], AT(0));
            __syncthreads();
            const int nr = (int)(re - rs);
            int tpr = 1;
            while (tpr < 64 && tpr * 2 * nr <= BLOCK) tpr <<= 1;
            const int row = tid / tpr, lane = tid & (tpr - 1);
            AT s = AT(0);
            if (row < nr) {
                const int b0 = (int)(rp[rs + row] - ps), e0 = (int)(rp[rs + row + 1] - ps);
                for (int k = b0 + lane; k < e0; k += tpr) s += prod[k];
            }
            for (int o = tpr >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (row < nr && lane == 0) epilogue(rs + row, (double)s);
            __syncthreads();
        } else {
            const int lid = -1 - item.x;
            const int64_t r = lrow[lid];
            const int64_t p0 = rp[r] + (int64_t)item.y * CH;
            const int64_t p1 = min(p0 + (int64_t)CH, rp[r + 1]);
            AT s = AT(0);
            for (int64_t p = p0 + tid; p < p1; p += BLOCK) s += to_a(val[p], AT(0)) * to_a(x[col[p]], AT(0));
            s = block_sum(s, sha);
            if (tid == 0) lpart[it] = (double)s;
            if (last_block(&ltk[lid], (uint32_t)lnch[lid], &s_last)) {
                if (tid == 0) {
                    const int f = lfirst[lid], nc = lnch[lid];
                    double tot = 0.0;
                    for (int q = 0; q < nc; ++q) tot += lpart[f + q];
                    if (EPI == EPI_LANCZOS) {
                        const double y = sj * tot;
                        lval[lid] = sj * to_d(x[r]) * y;
                        const double wp = xp ? bsc * to_d(xp[r]) : 0.0;
                        w[r] = (WT)(y - wp);
                    } else {
                        w[r] = (WT)tot;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (EPI != EPI_LANCZOS) return;
    apart = block_sum(apart, shd);
    if (tid == 0) part[blockIdx.x] = apart;
    if (last_block(&st->ticket[TK_SPMV], gridDim.x, &s_last)) {
        const double a = ordered_sum(part, gridDim.x, shd);
        const double al = ordered_sum(lval, st->n_long, shd);
        if (tid == 0) {
            const double alpha = a + al;
            st->alpha[j] = alpha;
            if (st->reorth == 0) {          // three-term recurrence only
                st->c2[j] = alpha;
                st->second = 1;
            }
        }
    }
}

// ------------------------------------------------- reorthogonalisation
// Active-kernel rules: the dot pass runs unless reorthogonalisation is off;
// the fused update+dot runs for two-pass modes.  A restart vector is always
// orthogonalised twice.
__device__ __forceinline__ bool dot_active(const State* st) {
    return st->reorth != 0 || st->mode == MODE_RESTART;
}
__device__ __forceinline__ bool upd_dot_active(const State* st) {
    return st->reorth >= 2 || st->mode == MODE_RESTART;
}

// c = V[:,0..j]^T w (coefficients with respect to the unit basis vectors).
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_orth_dot(State* st, const typename Tr<P>::V* __restrict__ Vb,
                                                    const typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                    double* part) {
    __shared__ double red[4][NC];
    __shared__ double shc[4][64];
    __shared__ int s_last;
    const int j = st->j;
    if (j >= st->m || !dot_active(st)) return;
    const int nc = j + 1;
    if (nc > NC) {                       // launch contract broken: flag, do nothing
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK) {
        const double wr = (double)w[r];
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k < nc) acc[k] += to_d(Vb[(int64_t)k * ld + r]) * wr;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < nc) {
            const double v = wave_sum(acc[k]);
            if (ln == 0) red[wv][k] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < nc)
        part[(int64_t)blockIdx.x * NCMAX + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    if (last_block(&st->ticket[TK_DOT], gridDim.x, &s_last)) {
        reduce_columns(part, gridDim.x, nc, st->scale, st->c, shc);
        if (threadIdx.x == 0 && !upd_dot_active(st)) st->second = 1;   // one pass: store step uses c
        __syncthreads();
        if (!upd_dot_active(st))
            for (int k = threadIdx.x; k < nc; k += BLOCK) st->c2[k] = st->c[k];
    }
}

// w' = w - V c (stored in the working precision), then c2 = V^T w' and ||w'||^2.
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_orth_upd_dot(State* st, const typename Tr<P>::V* __restrict__ Vb,
                                                        typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                        double* part, double* part2) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    __shared__ double cs[NC];
    __shared__ double red[4][NC];
    __shared__ double shc[4][64];
    __shared__ double shd[4];
    __shared__ int s_last;
    const int j = st->j;
    if (j >= st->m || !upd_dot_active(st)) return;
    const int nc = j + 1;
    if (nc > NC) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    for (int k = threadIdx.x; k < NC; k += BLOCK) cs[k] = k < nc ? st->c[k] * st->scale[k] : 0.0;
    __syncthreads();
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    double nrm = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK) {
        VT v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = k < nc ? Vb[(int64_t)k * ld + r] : VT(0);
        double x = (double)w[r];
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k < nc) x -= to_d(v[k]) * cs[k];
        const WT xw = (WT)x;
        w[r] = xw;
        const double xr = (double)xw;
        nrm += xr * xr;
#pragma unroll
        for (int k = 0; k < NC; ++k)
            if (k < nc) acc[k] += to_d(v[k]) * xr;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < nc) {
            const double v = wave_sum(acc[k]);
            if (ln == 0) red[wv][k] = v;
        }
    nrm = block_sum(nrm, shd);
    if ((int)threadIdx.x < nc)
        part[(int64_t)blockIdx.x * NCMAX + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    if (threadIdx.x == 0) part2[blockIdx.x] = nrm;
    if (last_block(&st->ticket[TK_UPD], gridDim.x, &s_last)) {
        reduce_columns(part, gridDim.x, nc, st->scale, st->c2, shc);
        const double wn = ordered_sum(part2, gridDim.x, shd);
        if (threadIdx.x == 0) {
            st->wnorm2 = wn;
            int second = 1;
            if (st->reorth == 3 && st->mode != MODE_RESTART) {
                // Selective: skip the second update when its correction is
                // below the rounding of the stored vector.
                double c2n = 0.0;
                for (int k = 0; k < nc; ++k) c2n += st->c2[k] * st->c2[k];
                second = c2n > st->u_s * st->u_s * wn;
            }
            st->second = second;
        }
    }
}

// v_{j+1} = w' - V c2 (if the second update runs), stored in the basis
// precision into column j+1; beta_{j+1} = ||stored column||; breakdown check.
template <int P, int NC>
__global__ __launch_bounds__(BLOCK) void k_orth_upd_store(State* st, typename Tr<P>::V* __restrict__ Vb,
                                                          const typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                          double* part2) {
    using VT = typename Tr<P>::V;
    __shared__ double cs[NC];
    __shared__ double shd[4];
    __shared__ int s_last;
    const int j = st->j;
    if (j >= st->m) return;
    const int nc = j + 1;
    if (nc > NC) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    const bool second = st->second != 0;
    const int lo = (st->reorth == 0 && st->mode != MODE_RESTART) ? j : 0;
    for (int k = threadIdx.x; k < NC; k += BLOCK)
        cs[k] = (second && k >= lo && k < nc) ? st->c2[k] * st->scale[k] : 0.0;
    __syncthreads();
    VT* out = Vb + (int64_t)(j + 1) * ld;
    double nrm = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK) {
        double x = (double)w[r];
        if (second) {
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (k >= lo && k < nc) x -= to_d(Vb[(int64_t)k * ld + r]) * cs[k];
        }
        const VT v = from_d<VT>(x);
        out[r] = v;
        const double d = to_d(v);
        nrm += d * d;
    }
    nrm = block_sum(nrm, shd);
    if (threadIdx.x == 0) part2[blockIdx.x] = nrm;
    if (last_block(&st->ticket[TK_STORE], gridDim.x, &s_last)) {
        const double tot = ordered_sum(part2, gridDim.x, shd);
        if (threadIdx.x == 0) {
            const double b = sqrt(tot);
            if (!isfinite(b)) {
                st->status = -7;               // LZ_ERR_NONFINITE
                st->j = st->m;
            } else if (st->mode == MODE_NORMAL) {
                const double t = fabs(st->alpha[j]) + st->beta[j];
                if (t > st->tnorm) st->tnorm = t;
                const double tau = 100.0 * st->u_s * st->tnorm;
                if (!(b > tau) && j + 1 < st->m) {
                    // Breakdown: the Krylov space is invariant.  T gets a zero
                    // coupling and the next iteration draws a restart vector.
                    st->mode = MODE_RESTART;
                    st->restarts += 1;
                    st->beta[j + 1] = 0.0;
                } else {
                    st->beta[j + 1] = b;
                    st->scale[j + 1] = b > 0.0 ? 1.0 / b : 0.0;
                    st->j = j + 1;
                }
            } else {
                if (!(b > 0.0)) {
                    st->status = -8;           // LZ_ERR_BREAKDOWN
                    st->j = st->m;
                } else {
                    st->scale[j + 1] = 1.0 / b;
                    st->beta[j + 1] = 0.0;
                    st->mode = MODE_NORMAL;
                    st->j = j + 1;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- Jacobi
// Parallel cyclic Jacobi on T (Sec. II, second phase) in one workgroup, in
// LDS.  Each round applies m/2 disjoint rotations chosen by the round-robin
// tournament ordering; m-1 rounds make a sweep.  Rotation (Rutishauser):
// zeta = (t_qq - t_pp)/(2 t_pq), t = sgn(zeta)/(|zeta| + sqrt(1+zeta^2)),
// c = 1/sqrt(1+t^2), s = t c.  A rotation is skipped when |t_pq| is
// negligible (<= eps sqrt|t_pp t_qq| or <= eps^2 ||T||_F); the method stops
// after a sweep without rotations.  Then Top-K by modulus (Sec. I).
constexpr int JMAX_SWEEPS = 60;

__device__ void jacobi_core(int m, double (*T)[MMAX + 1], double (*S)[MMAX + 1], double fro, int* sweeps_out,
                            int* rot_flag) {
    __shared__ double rc[MMAX / 2], rs[MMAX / 2];
    __shared__ int rp_[MMAX / 2], rq_[MMAX / 2];
    const double eps = 1.1102230246251565e-16;
    const int me = (m + 1) & ~1;           // even number of players (one dummy if m is odd)
    const int half = me / 2;
    int sweeps = -1;
    for (int sweep = 1; sweep <= JMAX_SWEEPS; ++sweep) {
        if (threadIdx.x == 0) *rot_flag = 0;
        __syncthreads();
        for (int round = 0; round < me - 1; ++round) {
            if ((int)threadIdx.x < half) {
                const int i = threadIdx.x;
                auto pos = [&](int k) { return k == 0 ? 0 : 1 + ((k - 1 + round) % (me - 1)); };
                int p = pos(i), q = pos(me - 1 - i);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                bool rot = false;
                if (q < m) {
                    const double apq = T[p][q], app = T[p][p], aqq = T[q][q];
                    if (!(fabs(apq) <= eps * sqrt(fabs(app * aqq)) || fabs(apq) <= eps * eps * fro)) {
                        const double zeta = (aqq - app) / (2.0 * apq);
                        double t;
                        if (fabs(zeta) > 1e150)
                            t = 0.5 / zeta;
                        else
                            t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        rot = true;
                    }
                }
                rc[i] = c;
                rs[i] = s;
                rp_[i] = rot ? p : -1;
                rq_[i] = q;
                if (rot) *rot_flag = 1;
            }
            __syncthreads();
            // Rows p, q of T  <-  J^T T
            for (int idx = threadIdx.x; idx < half * m; idx += BLOCK) {
                const int i = idx / m, cc = idx % m;
                const int p = rp_[i];
                if (p < 0) continue;
                const int q = rq_[i];
                const double tp = T[p][cc], tq = T[q][cc];
                T[p][cc] = rc[i] * tp - rs[i] * tq;
                T[q][cc] = rs[i] * tp + rc[i] * tq;
            }
            __syncthreads();
            // Columns p, q of T and S  <-  T J, S J
            for (int idx = threadIdx.x; idx < half * m; idx += BLOCK) {
                const int i = idx / m, rr = idx % m;
                const int p = rp_[i];
                if (p < 0) continue;
                const int q = rq_[i];
                const double tp = T[rr][p], tq = T[rr][q];
                T[rr][p] = rc[i] * tp - rs[i] * tq;
                T[rr][q] = rs[i] * tp + rc[i] * tq;
                const double sp = S[rr][p], sq = S[rr][q];
                S[rr][p] = rc[i] * sp - rs[i] * sq;
                S[rr][q] = rs[i] * sp + rc[i] * sq;
            }
            __syncthreads();
            if ((int)threadIdx.x < half && rp_[threadIdx.x] >= 0) {
                T[rp_[threadIdx.x]][rq_[threadIdx.x]] = 0.0;
                T[rq_[threadIdx.x]][rp_[threadIdx.x]] = 0.0;
            }
            __syncthreads();
        }
        const int any = *rot_flag;
        __syncthreads();
        if (!any) {
            sweeps = sweep;
            break;
        }
    }
    *sweeps_out = sweeps;
}

// Builds T from the Lanczos coefficients, diagonalises it, selects the
// Top-K and writes the eigenvalues.
__global__ __launch_bounds__(BLOCK) void k_jacobi_select(State* st, double* out_vals) {
    __shared__ double T[MMAX][MMAX + 1];
    __shared__ double S[MMAX][MMAX + 1];
    __shared__ double shd[4];
    __shared__ int rot_flag, sweeps;
    if (st->status != 0) return;
    const int m = min(st->j, st->m);
    const int K = st->K;
    if (m < K) {
        if (threadIdx.x == 0) st->status = -8;
        return;
    }
    double f = 0.0;
    for (int idx = threadIdx.x; idx < m * m; idx += BLOCK) {
        const int r = idx / m, c = idx % m;
        double t = 0.0;
        if (r == c) t = st->alpha[r];
        else if (c == r + 1) t = st->beta[c];
        else if (r == c + 1) t = st->beta[r];
        T[r][c] = t;
        S[r][c] = r == c ? 1.0 : 0.0;
        f += t * t;
    }
    f = block_sum(f, shd);
    __syncthreads();
    jacobi_core(m, T, S, sqrt(f), &sweeps, &rot_flag);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += BLOCK) st->theta[i] = T[i][i];
    for (int idx = threadIdx.x; idx < m * m; idx += BLOCK) st->S[(idx / m) * MMAX + idx % m] = S[idx / m][idx % m];
    // Rank of each Ritz value in the order |theta| desc, theta desc, index asc.
    for (int i = threadIdx.x; i < m; i += BLOCK) {
        const double ti = T[i][i];
        int rank = 0;
        for (int k = 0; k < m; ++k) {
            const double tk = T[k][k];
            const bool before = fabs(tk) > fabs(ti) || (fabs(tk) == fabs(ti) && (tk > ti || (tk == ti && k < i)));
            rank += before;
        }
        if (rank < K) {
            st->sel[rank] = i;
            if (out_vals) out_vals[rank] = ti;
        }
    }
    if (threadIdx.x == 0) {
        st->sweeps = sweeps;
        if (sweeps < 0) st->status = -6;       // LZ_ERR_NOT_CONVERGED
    }
}

// Standalone tridiagonal eigensolve (component entry point).
__global__ __launch_bounds__(BLOCK) void k_jacobi_only(const double* alpha, const double* offd, int m, State* st) {
    __shared__ double T[MMAX][MMAX + 1];
    __shared__ double S[MMAX][MMAX + 1];
    __shared__ double shd[4];
    __shared__ int rot_flag, sweeps;
    double f = 0.0;
    for (int idx = threadIdx.x; idx < m * m; idx += BLOCK) {
        const int r = idx / m, c = idx % m;
        double t = 0.0;
        if (r == c) t = alpha[r];
        else if (c == r + 1) t = offd[r];
        else if (r == c + 1) t = offd[c];
        T[r][c] = t;
        S[r][c] = r == c ? 1.0 : 0.0;
        f += t * t;
    }
    f = block_sum(f, shd);
    __syncthreads();
    jacobi_core(m, T, S, sqrt(f), &sweeps, &rot_flag);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += BLOCK) st->theta[i] = T[i][i];
    for (int idx = threadIdx.x; idx < m * m; idx += BLOCK) st->S[(idx / m) * MMAX + idx % m] = S[idx / m][idx % m];
    if (threadIdx.x == 0) {
        st->sweeps = sweeps;
        st->status = sweeps < 0 ? -6 : 0;
    }
}

// ------------------------------------------------------------ Ritz vectors
// Y[r, k] = sum_i scale_i V[r, i] S[i, sel_k]  (Sec. II: eigenvectors of the
// matrix are the Lanczos basis times those of T); Y is row-major n x K.
template <int P, int KB>
__global__ __launch_bounds__(BLOCK) void k_ritz(State* st, const typename Tr<P>::V* __restrict__ Vb, int64_t n,
                                                int64_t ld, double* __restrict__ Y) {
    __shared__ double Ss[MMAX][KB];
    if (st->status != 0) return;
    const int m = min(st->j, st->m), K = st->K;
    for (int idx = threadIdx.x; idx < MMAX * KB; idx += BLOCK) {
        const int i = idx / KB, k = idx % KB;
        Ss[i][k] = (i < m && k < K) ? st->S[i * MMAX + st->sel[k]] * st->scale[i] : 0.0;
    }
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLOCK) {
        double acc[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) acc[k] = 0.0;
        for (int i = 0; i < m; ++i) {
            const double v = to_d(Vb[(int64_t)i * ld + r]);
#pragma unroll
            for (int k = 0; k < KB; ++k) acc[k] += v * Ss[i][k];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (k < K) Y[r * K + k] = acc[k];
    }
}

// Per column k of Y: norm and the entry of largest modulus (lowest row on
// ties) -> ysc[k] = sign(that entry) / norm.  Lane k of each group of KB lanes
// owns column k.
__global__ __launch_bounds__(BLOCK) void k_colstats(State* st, const double* __restrict__ Y, int64_t n, int KB,
                                                    double* part) {
    __shared__ double s_n[BLOCK], s_a[BLOCK], s_v[BLOCK];
    __shared__ int64_t s_i[BLOCK];
    __shared__ int s_last;
    if (st->status != 0) return;
    const int K = st->K;
    const int groups = BLOCK / KB, g = threadIdx.x / KB, k = threadIdx.x % KB;
    double nrm = 0.0, best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    if (k < K) {
        for (int64_t r = (int64_t)blockIdx.x * groups + g; r < n; r += (int64_t)gridDim.x * groups) {
            const double y = Y[r * K + k];
            nrm += y * y;
            const double a = fabs(y);
            if (a > best || (a == best && r < bidx)) { best = a; bval = y; bidx = r; }
        }
    }
    s_n[threadIdx.x] = nrm; s_a[threadIdx.x] = best; s_v[threadIdx.x] = bval; s_i[threadIdx.x] = bidx;
    __syncthreads();
    if ((int)threadIdx.x < KB) {
        double tn = 0.0, ta = -1.0, tv = 0.0;
        int64_t ti = INT64_MAX;
        for (int gg = 0; gg < groups; ++gg) {
            const int t = gg * KB + threadIdx.x;
            tn += s_n[t];
            if (s_a[t] > ta || (s_a[t] == ta && s_i[t] < ti)) { ta = s_a[t]; tv = s_v[t]; ti = s_i[t]; }
        }
        double* pb = part + (int64_t)blockIdx.x * 4 * 64;
        pb[threadIdx.x] = tn;
        pb[64 + threadIdx.x] = ta;
        pb[128 + threadIdx.x] = tv;
        pb[192 + threadIdx.x] = (double)ti;
    }
    if (last_block(&st->ticket[TK_RITZ], gridDim.x, &s_last)) {
        if ((int)threadIdx.x < K) {
            double tn = 0.0, ta = -1.0, tv = 0.0, ti = 1e300;
            for (unsigned b = 0; b < gridDim.x; ++b) {
                const double* pb = part + (int64_t)b * 4 * 64;
                tn += pb[threadIdx.x];
                const double a = pb[64 + threadIdx.x], i = pb[192 + threadIdx.x];
                if (a > ta || (a == ta && i < ti)) { ta = a; tv = pb[128 + threadIdx.x]; ti = i; }
            }
            st->ysc[threadIdx.x] = (tv < 0.0 ? -1.0 : 1.0) / sqrt(tn);
        }
    }
}

// Residual report and output (Sec. IV-D): for each row r and Ritz pair k,
// d = (A y_k)[r] - theta_k y_k[r] with y_k = ysc_k Y[:,k]; accumulates d^2
// and writes out_vecs[k*n + r] = y_k[r].  Lane k of a group of KB lanes
// owns pair k; a group walks one row's non-zeros, reading K-wide rows of Y.
__global__ __launch_bounds__(BLOCK) void k_resid_out(State* st, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col, const void* valp, int prec,
                                                     const double* __restrict__ Y, int64_t n, int KB,
                                                     const int2* __restrict__ items, const int32_t* lrow,
                                                     const int32_t* lfirst, const int32_t* lnch, uint32_t* ltk,
                                                     double* lpart, double* lval, double* part, double* out_vecs,
                                                     int do_resid) {
    __shared__ double sred[BLOCK];
    __shared__ double shk[BLOCK];
    __shared__ int s_last;
    if (st->status != 0) return;
    const int K = st->K;
    const int groups = BLOCK / KB, g = threadIdx.x / KB, k = threadIdx.x % KB;
    const bool act = k < K;
    const double ysc = act ? st->ysc[k] : 0.0;
    const double th = act ? st->theta[st->sel[k]] : 0.0;
    auto vload = [&](int64_t p) -> double {
        if (prec == 0) return ((const double*)valp)[p];
        if (prec == 1) return (double)((const float*)valp)[p];
        return (double)__uint_as_float((uint32_t)((const uint16_t*)valp)[p] << 16);
    };
    double racc = 0.0;
    const int nitems = st->n_items;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        if (item.x >= 0) {
            for (int64_t r = item.x + g; r < item.y; r += groups) {
                double z = 0.0;
                if (act && do_resid)
                    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) z += vload(p) * Y[(int64_t)col[p] * K + k];
                if (act) {
                    const double y = ysc * Y[r * K + k];
                    out_vecs[(int64_t)k * n + r] = y;
                    const double d = ysc * z - th * y;
                    racc += d * d;
                }
            }
        } else {
            const int lid = -1 - item.x;
            const int64_t r = lrow[lid];
            const int64_t p0 = rp[r] + (int64_t)item.y * CH;
            const int64_t p1 = min(p0 + (int64_t)CH, rp[r + 1]);
            double z = 0.0;
            if (act && do_resid)
                for (int64_t p = p0 + g; p < p1; p += groups) z += vload(p) * Y[(int64_t)col[p] * K + k];
            shk[threadIdx.x] = z;
            __syncthreads();
            if (g == 0 && act) {
                double s = 0.0;
                for (int gg = 0; gg < groups; ++gg) s += shk[gg * KB + k];
                lpart[(int64_t)it * KB + k] = s;
            }
            if (last_block(&ltk[lid], (uint32_t)lnch[lid], &s_last)) {
                if (g == 0 && act) {
                    const int f = lfirst[lid], nc = lnch[lid];
                    double tot = 0.0;
                    for (int q = 0; q < nc; ++q) tot += lpart[(int64_t)(f + q) * KB + k];
                    const double y = ysc * Y[r * K + k];
                    out_vecs[(int64_t)k * n + r] = y;
                    const double d = ysc * tot - th * y;
                    lval[(int64_t)lid * KB + k] = d * d;
                }
            }
            __syncthreads();
        }
    }
    // Per-pair partial sums over the workgroup's groups, in group order.
    sred[threadIdx.x] = racc;
    __syncthreads();
    if ((int)threadIdx.x < KB) {
        double s = 0.0;
        for (int gg = 0; gg < groups; ++gg) s += sred[gg * KB + threadIdx.x];
        part[(int64_t)blockIdx.x * 64 + threadIdx.x] = s;
    }
    if (last_block(&st->ticket[TK_RESID], gridDim.x, &s_last)) {
        if ((int)threadIdx.x < K) {
            double s = 0.0;
            for (unsigned b = 0; b < gridDim.x; ++b) s += part[(int64_t)b * 64 + threadIdx.x];
            const int nl = st->n_long;
            for (int l = 0; l < nl; ++l) s += lval[(int64_t)l * KB + threadIdx.x];
            const double a = sqrt(s);
            st->abs_resid[threadIdx.x] = a;
            st->resid[threadIdx.x] = th != 0.0 ? a / fabs(th) : a;
        }
    }
}

// ---------------------------------------------------------------- launchers
static inline int nc_bucket(int ncols) { return ((ncols + 7) / 8) * 8; }

template <int P>
static hipError_t iteration_p(const Plan& p, const Bufs& b, const Csr& a, int ncols, hipStream_t s) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    VT* V = (VT*)b.V;
    WT* w = (WT*)b.w;
    hipLaunchKernelGGL((k_spmv<P, EPI_LANCZOS>), dim3(p.g_spmv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                       (const VT*)a.val, V, w, a.n, p.ld, b.items, b.lrow, b.lfirst, b.lnch, b.ltk, b.lpart,
                       b.lval, b.part2);
    const int nb = nc_bucket(ncols);
#define LZ_ORTH_CASE(NCV)                                                                                  \
    case NCV:                                                                                              \
        hipLaunchKernelGGL((k_orth_dot<P, NCV>), dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, V, w, p.ld,      \
                           b.part);                                                                        \
        hipLaunchKernelGGL((k_orth_upd_dot<P, NCV>), dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, V, w, p.ld,  \
                           b.part, b.part2);                                                               \
        hipLaunchKernelGGL((k_orth_upd_store<P, NCV>), dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, V, w,     \
                           p.ld, b.part2);                                                                 \
        break;
    switch (nb) {
        LZ_ORTH_CASE(8)
        LZ_ORTH_CASE(16)
        LZ_ORTH_CASE(24)
        LZ_ORTH_CASE(32)
        LZ_ORTH_CASE(40)
        LZ_ORTH_CASE(48)
        LZ_ORTH_CASE(56)
        LZ_ORTH_CASE(64)
        LZ_ORTH_CASE(72)
        default:
            return hipErrorInvalidValue;
    }
#undef LZ_ORTH_CASE
    return hipGetLastError();
}

hipError_t launch_iteration(const Plan& p, const Bufs& b, const Csr& a, int ncols, hipStream_t s) {
    switch (p.prec) {
        case 0: return iteration_p<0>(p, b, a, ncols, s);
        case 1: return iteration_p<1>(p, b, a, ncols, s);
        case 2: return iteration_p<2>(p, b, a, ncols, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_setup(const Plan& p, const Bufs& b, const Csr& a, uint64_t seed, int reorth, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(BLOCK), 0, s, b.st, p.m, p.K, reorth, unit_roundoff(p.prec), seed);
    const int64_t n = a.n;
    const int g = (int)std::min<int64_t>((n + BLOCK - 1) / BLOCK, 8192);
    const int gv = (int)std::min<int64_t>((std::max(n, a.nnz) + BLOCK - 1) / BLOCK, 8192);
    hipLaunchKernelGGL(k_validate, dim3(gv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col, n, a.nnz);
    hipLaunchKernelGGL(k_setup_count, dim3(g), dim3(BLOCK), 0, s, a.rowptr, n, b.scan);
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(BLOCK), 0, s, b.scan, n, b.bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, s, b.bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(BLOCK), 0, s, b.scan, n, b.bsum);
    hipLaunchKernelGGL(k_setup_items, dim3(g), dim3(BLOCK), 0, s, a.rowptr, n, b.scan, b.bsum + nb, p.items_cap,
                       p.long_cap, b.items, b.lrow, b.lfirst, b.lnch, b.ltk, b.st);
    return hipGetLastError();
}

hipError_t launch_init(const Plan& p, const Bufs& b, hipStream_t s) {
    switch (p.prec) {
        case 0:
            hipLaunchKernelGGL(k_init<0>, dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, (double*)b.V, (double*)b.w, p.n,
                               p.ld, b.part2);
            break;
        case 1:
            hipLaunchKernelGGL(k_init<1>, dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, (float*)b.V, (float*)b.w, p.n,
                               p.ld, b.part2);
            break;
        case 2:
            hipLaunchKernelGGL(k_init<2>, dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, (uint16_t*)b.V, (float*)b.w,
                               p.n, p.ld, b.part2);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int P>
static hipError_t ritz_p(const Plan& p, const Bufs& b, hipStream_t s) {
    using VT = typename Tr<P>::V;
    const VT* V = (const VT*)b.V;
    const int g = p.g_orth;
    switch (p.KB) {
#define LZ_RITZ_CASE(KBV)                                                                                    \
    case KBV:                                                                                                \
        hipLaunchKernelGGL((k_ritz<P, KBV>), dim3(g), dim3(BLOCK), 0, s, b.st, V, p.n, p.ld, b.Y);         \
        break;
        LZ_RITZ_CASE(8)
        LZ_RITZ_CASE(16)
        LZ_RITZ_CASE(24)
        LZ_RITZ_CASE(32)
        LZ_RITZ_CASE(40)
        LZ_RITZ_CASE(48)
        LZ_RITZ_CASE(56)
        LZ_RITZ_CASE(64)
#undef LZ_RITZ_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static int pow2_at_least(int k) {
    int v = 1;
    while (v < k) v <<= 1;
    return v;
}

hipError_t launch_finish(const Plan& p, const Bufs& b, const Csr& a, double* out_vals, double* out_vecs, int report,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_select, dim3(1), dim3(BLOCK), 0, s, b.st, out_vals);
    hipError_t e = hipSuccess;
    switch (p.prec) {
        case 0: e = ritz_p<0>(p, b, s); break;
        case 1: e = ritz_p<1>(p, b, s); break;
        case 2: e = ritz_p<2>(p, b, s); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const int kb2 = pow2_at_least(p.K);
    hipLaunchKernelGGL(k_colstats, dim3(p.g_orth), dim3(BLOCK), 0, s, b.st, b.Y, p.n, kb2, b.part);
    hipLaunchKernelGGL(k_resid_out, dim3(p.g_spmv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col, a.val, p.prec, b.Y,
                       p.n, kb2, b.items, b.lrow, b.lfirst, b.lnch, b.ltk, b.lpart, b.lval, b.part2, out_vecs,
                       report);
    return hipGetLastError();
}

hipError_t launch_spmv_plain(const Plan& p, const Bufs& b, const Csr& a, const void* x, void* y, hipStream_t s) {
    switch (p.prec) {
        case 0:
            hipLaunchKernelGGL((k_spmv<0, EPI_PLAIN>), dim3(p.g_spmv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                               (const double*)a.val, (const double*)x, (double*)y, a.n, p.ld, b.items, b.lrow,
                               b.lfirst, b.lnch, b.ltk, b.lpart, b.lval, b.part2);
            break;
        case 1:
            hipLaunchKernelGGL((k_spmv<1, EPI_PLAIN>), dim3(p.g_spmv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                               (const float*)a.val, (const float*)x, (float*)y, a.n, p.ld, b.items, b.lrow,
                               b.lfirst, b.lnch, b.ltk, b.lpart, b.lval, b.part2);
            break;
        case 2:
            hipLaunchKernelGGL((k_spmv<2, EPI_PLAIN>), dim3(p.g_spmv), dim3(BLOCK), 0, s, b.st, a.rowptr, a.col,
                               (const uint16_t*)a.val, (const uint16_t*)x, (float*)y, a.n, p.ld, b.items, b.lrow,
                               b.lfirst, b.lnch, b.ltk, b.lpart, b.lval, b.part2);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_jacobi_only(const double* alpha, const double* offdiag, int m, State* st, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_only, dim3(1), dim3(BLOCK), 0, s, alpha, offdiag, m, st);
    return hipGetLastError();
}

}  // namespace lz
