// gfx950 kernels of one Lanczos iteration (Sec. III, Algorithm 1) and the
// start vector.
//
// One iteration is three kernels:
//   k_spmv_step      w = A v_j - beta_j v_{j-1};  alpha_j = v_j . (A v_j)
//   k_orth_dot       c = V^T w; the second Gram-Schmidt coefficients
//                    c2 = V^T (w - V c) = c - G c from the Gram matrix G of
//                    the stored basis (no second pass over V)
//   k_orth_upd_store v_{j+1} = w - V (c + c2) in the basis precision;
//                    beta_{j+1}; the new column of G
// With one pass or none, a restart vector (always orthogonalised twice) takes
// the classical second pass instead: k_orth_upd_dot, w' = w - V c and
// c2 = V^T w', runs between the two.  The two-pass modes run it too when the
// first pass cancelled strongly (see k_orth_dot).
// Global sums are per-workgroup partials that the last workgroup to finish
// adds in a fixed order, so results do not depend on scheduling.  The step
// index and every coefficient stay in device memory.
//
// The basis V is column-major with leading dimension ld (a multiple of
// LDPAD); rows n..ld-1 stay zero so the dense kernels need no tail handling.
// Column k is stored unnormalised; scale[k] makes it unit length.
#include <algorithm>
#include <cmath>

#include "lz_spmv.h"

namespace lz {

// ------------------------------------------------------------ start vector
// V[:,0] = u rounded to the basis precision, u_r = U01(SplitMix64(seed, r))
// with r the original row index; scale[0] = 1/||stored u||.  Also clears w
// (its padding rows must stay zero).
template <int P>
__global__ __launch_bounds__(BLOCK) void k_init(State* st, typename Tr<P>::V* V, typename Tr<P>::W* w,
                                                int64_t n, int64_t ld, double* part, double* gm) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    __shared__ double sh[BLOCK / 64];
    __shared__ int s_last;
    if (st->status != 0) {                 // invalid input: no Lanczos step will run
        if (blockIdx.x == 0 && threadIdx.x == 0) st->j = st->m;
        return;
    }
    const uint64_t seed = st->seed;
    const int32_t* perm = st->perm;
    double s = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < ld; r += (int64_t)gridDim.x * BLOCK) {
        const VT v = from_d<VT>(r < n ? u01(seed, (uint64_t)(perm ? perm[r] : r)) : 0.0);
        V[r] = v;
        w[r] = (WT)0;
        const double d = to_d(v);
        s += d * d;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) st_dev(&part[blockIdx.x], s);
    if (last_block(&st->ticket[TK_INIT], gridDim.x, &s_last)) {
        const double tot = ordered_sum_dev(part, gridDim.x, sh);
        if (threadIdx.x == 0) {
            if (st->arith) {               // all-FP32 mode: the norm's square root and scale in FP32
                const float sc = 1.0f / sqrtf((float)tot);
                st->scale[0] = sc;
                gm[0] = (double)((float)tot * sc * sc);
            } else {
                st->scale[0] = 1.0 / sqrt(tot);
                gm[0] = tot * st->scale[0] * st->scale[0];
            }
            st->beta[0] = 0.0;
            st->j = 0;
            st->mode = MODE_NORMAL;
        }
    }
}

// ------------------------------------------------- reorthogonalisation
// The dot pass runs unless reorthogonalisation is off.  The two-pass modes
// keep the Gram matrix of the stored basis and take the second coefficients
// from it; the one-pass modes run the classical second pass only for a
// restart vector (always orthogonalised twice).
__device__ __forceinline__ bool dot_active(const State* st) {
    return st->reorth != 0 || st->mode == MODE_RESTART;
}
__device__ __forceinline__ bool gram_mode(const State* st) { return st->reorth >= 2; }
__device__ __forceinline__ bool upd_dot_active(const State* st) {
    return gram_mode(st) ? st->remeasure != 0 : st->mode == MODE_RESTART;
}

// The dense kernels move 16-byte chunks: R consecutive rows of one basis
// column (2 in FP64, 4 in FP32, 8 in BF16) and the matching R rows of w.
// The columns of a step are split over CS adjacent lanes (NCL each), so a
// lane keeps at most 8 chunks in registers; CS lanes together own a row
// group and combine their partial updates with shuffles.
template <int P> struct Ch;
template <> struct Ch<0> { typedef double2 T; static constexpr int R = 2; };
template <> struct Ch<1> { typedef float4 T; static constexpr int R = 4; };
template <> struct Ch<2> { typedef uint4 T; static constexpr int R = 8; };

template <int P, int NC> struct Split {
    static constexpr int NCLMAX = 8;                   // chunks a lane keeps in registers
    static constexpr int CS = NC <= NCLMAX ? 1 : (NC <= 2 * NCLMAX ? 2 : (NC <= 4 * NCLMAX ? 4 : 8));
    static constexpr int NCL = NC / CS;
};

// Keeps the compiler from holding widened copies of the packed chunks
// between the update and the dot pass (they are re-widened instead).
__device__ __forceinline__ void opaque(double2& c) { asm volatile("" : "+v"(c.x), "+v"(c.y)); }
__device__ __forceinline__ void opaque(float4& c) { asm volatile("" : "+v"(c.x), "+v"(c.y), "+v"(c.z), "+v"(c.w)); }
__device__ __forceinline__ void opaque(uint4& c) { asm volatile("" : "+v"(c.x), "+v"(c.y), "+v"(c.z), "+v"(c.w)); }

__device__ __forceinline__ void unpack(const double2& c, double (&o)[2]) { o[0] = c.x; o[1] = c.y; }
template <class A>
__device__ __forceinline__ void unpack(const float4& c, A (&o)[4]) {
    o[0] = c.x; o[1] = c.y; o[2] = c.z; o[3] = c.w;
}
__device__ __forceinline__ double bf_lo(uint32_t u) { return (double)__uint_as_float(u << 16); }
__device__ __forceinline__ double bf_hi(uint32_t u) { return (double)__uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ void unpack(const uint4& c, double (&o)[8]) {
    o[0] = bf_lo(c.x); o[1] = bf_hi(c.x); o[2] = bf_lo(c.y); o[3] = bf_hi(c.y);
    o[4] = bf_lo(c.z); o[5] = bf_hi(c.z); o[6] = bf_lo(c.w); o[7] = bf_hi(c.w);
}

// R rows of the working vector w.
__device__ __forceinline__ void w_load(const double* w, double (&o)[2]) { unpack(*(const double2*)w, o); }
template <class A>
__device__ __forceinline__ void w_load(const float* w, A (&o)[4]) { unpack(*(const float4*)w, o); }
__device__ __forceinline__ void w_load(const float* w, double (&o)[8]) {
    const float4 a = *(const float4*)w, b = *((const float4*)w + 1);
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w; o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
// Round x to the working precision in place; store when `st` is set.
__device__ __forceinline__ void w_round_store(double* w, double (&x)[2], bool st) {
    if (st) *(double2*)w = make_double2(x[0], x[1]);
}
template <class A>
__device__ __forceinline__ void w_round_store(float* w, A (&x)[4], bool st) {
    const float4 a = make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    if (st) *(float4*)w = a;
}
__device__ __forceinline__ void w_round_store(float* w, double (&x)[8], bool st) {
    const float4 a = make_float4((float)x[0], (float)x[1], (float)x[2], (float)x[3]);
    const float4 b = make_float4((float)x[4], (float)x[5], (float)x[6], (float)x[7]);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w; x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    if (st) {
        *(float4*)w = a;
        *((float4*)w + 1) = b;
    }
}
// Round x to the basis precision in place; store when `st` is set.
__device__ __forceinline__ void v_round_store(double* v, double (&x)[2], bool st) { w_round_store(v, x, st); }
template <class A>
__device__ __forceinline__ void v_round_store(float* v, A (&x)[4], bool st) { w_round_store(v, x, st); }
__device__ __forceinline__ void v_round_store(uint16_t* v, double (&x)[8], bool st) {
    uint32_t h[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        h[i] = f32_to_bf16((float)x[i]);
        x[i] = (double)__uint_as_float(h[i] << 16);
    }
    if (st) *(uint4*)v = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// The orthogonalisation kernels run workgroups of OBLOCK threads (OWAVES
// wavefronts), at most OGRID of them.  Each wavefront walks chunks of RBW =
// (64 / CS) * R rows (at most 512, so a chunk never crosses ld, a multiple of
// LDPAD), chunk index = global wavefront index, grid-strided.
constexpr int OWAVES = OBLOCK / 64;

// Wave sums of acc[kk] over the lanes that own the same columns (lane % CS
// equal); lanes 0..CS-1 write them to red[wave][column].  Then thread k < nc
// publishes the workgroup sum of column k (wavefronts in order) to
// part[blockIdx.x*NCMAX + k].
template <int NC, int CS, int NCL, class A>
__device__ __forceinline__ void publish_split(const A (&acc)[NCL], int nc, double* part, A (*red)[NC]) {
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, cs = ln % CS;
#pragma unroll
    for (int kk = 0; kk < NCL; ++kk) {
        A v = acc[kk];
#pragma unroll
        for (int o = CS; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
        if (ln < CS) red[wv][cs * NCL + kk] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        A s = red[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < OWAVES; ++q) s += red[q][threadIdx.x];
        st_dev(&part[(int64_t)blockIdx.x * NCMAX + threadIdx.x], (double)s);
    }
}

// Run by the last workgroup: out[k] = mul[k] * sum_b part[b*NCMAX + k] for
// k < nc over the nb <= OGRID workgroup rows; returns sum_b p2[b].  Thread t
// owns column t % (NC+1) (column NC stands for p2) in slice t / (NC+1), i.e.
// rows slice, slice + S, slice + 2S, ... (S slices).  Its loads do not depend
// on one another and are all issued before the first add, so the workgroup
// waits for one round of loads.  The S slice sums of a column are then added
// in slice order: the result depends on nb only, not on scheduling.
template <int NC, class A>
__device__ __forceinline__ A reduce_columns(const double* part, const double* p2, int nb, int nc,
                                            const double* mul, double* out, A* sred, A* sh) {
    constexpr int NCC = NC + 1, S = OBLOCK / NCC, RPT = (OGRID + S - 1) / S;
    static_assert(NC <= NCMAX && S >= 1, "column count");
    const int t = threadIdx.x, col = t % NCC, slice = t / NCC;
    if (slice < S) {
        const double* src = col < NC ? part + col : p2;
        const int64_t stride = col < NC ? NCMAX : 1;
        double v[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) v[i] = ld_dev(src + (int64_t)min(slice + i * S, nb - 1) * stride);
        A s = A(0);
#pragma unroll
        for (int i = 0; i < RPT; ++i) s += slice + i * S < nb ? (A)v[i] : A(0);
        sred[t] = s;
    }
    __syncthreads();
    if (t < NCC) {
        A s = sred[t];
        for (int q = 1; q < S; ++q) s += sred[q * NCC + t];
        if (t < nc) out[t] = (double)((A)mul[t] * s);
        if (t == NC) sh[0] = s;
    }
    __syncthreads();
    const A tot = sh[0];
    __syncthreads();
    return tot;
}

// c = V[:,0..j]^T w (coefficients with respect to the unit basis vectors).
// A is the arithmetic of the dots, norms and update: double, or float in the
// all-FP32 mode.
template <int P, int NC, class A>
__global__ __launch_bounds__(OBLOCK) void k_orth_dot(State* st, const typename Tr<P>::V* __restrict__ Vb,
                                                    const typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                    double* part, double* part2, const double* __restrict__ gm) {
    using VT = typename Tr<P>::V;
    using CT = typename Ch<P>::T;
    constexpr int R = Ch<P>::R, CS = Split<P, NC>::CS, NCL = Split<P, NC>::NCL, GPW = 64 / CS;
    __shared__ A red[OWAVES][NC];
    __shared__ A sc[NC];
    __shared__ A sg[NC][NC + 1];
    __shared__ A shd[OWAVES];
    __shared__ A sred[OBLOCK];
    __shared__ int s_last;
    const int j = st->j;
    if (st->status != 0 || j >= st->m || !dot_active(st)) return;
    const int nc = j + 1;
    if (nc > NC) {                       // launch contract broken: flag, do nothing
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    const int ln = threadIdx.x & 63, cs = ln % CS;
    constexpr int64_t RBW = (int64_t)GPW * R;
    const int64_t lane_row = (int64_t)(ln / CS) * R;
    const int64_t wave0 = (int64_t)blockIdx.x * OWAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    A acc[NCL];
#pragma unroll
    for (int kk = 0; kk < NCL; ++kk) acc[kk] = A(0);
    A nrm = A(0);
    for (int64_t base = wave0 * RBW; base < ld; base += (int64_t)gridDim.x * OWAVES * RBW) {
        const int64_t r0 = base + lane_row;
        A x[R];
        w_load(w + r0, x);
        if (cs == 0)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) nrm += x[rr] * x[rr];
        CT ch[NCL];
#pragma unroll
        for (int kk = 0; kk < NCL; ++kk) {
            const int k = cs * NCL + kk;
            if (k < nc) ch[kk] = *(const CT*)(Vb + (int64_t)k * ld + r0);
        }
#pragma unroll
        for (int kk = 0; kk < NCL; ++kk) {
            const int k = cs * NCL + kk;
            if (k < nc) {
                A v[R];
                unpack(ch[kk], v);
                A s = A(0);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) s += v[rr] * x[rr];
                acc[kk] += s;
            }
        }
    }
    publish_split<NC, CS, NCL>(acc, nc, part, red);
    nrm = block_sum(nrm, shd, OWAVES);
    if (threadIdx.x == 0) st_dev(&part2[blockIdx.x], (double)nrm);
    if (last_block(&st->ticket[TK_DOT], gridDim.x, &s_last)) {
        // The Gram rows the correction needs are loaded in the same round of
        // requests as the partials (nc^2 <= 4 * OBLOCK entries).
        const bool gram = gram_mode(st);
        A gv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = threadIdx.x + q * OBLOCK;
            gv[q] = (gram && idx < nc * nc) ? (A)gm[(idx / nc) * NCMAX + idx % nc] : A(0);
        }
        const A wn = reduce_columns<NC>(part, part2, gridDim.x, nc, st->scale, st->c, sred, shd);
        if (gram) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = threadIdx.x + q * OBLOCK;
                if (idx < nc * nc) sg[idx / nc][idx % nc] = gv[q];
            }
            // Second coefficients of classical Gram-Schmidt without a second
            // pass: V^T (w - V c) = c - G c, G the Gram matrix of the unit
            // stored basis.  The update then subtracts V (c + c2) at once, in
            // registers, so no rounded intermediate w' exists.
            for (int k = threadIdx.x; k < nc; k += OBLOCK) sc[k] = (A)st->c[k];
            __syncthreads();
            A c2 = A(0);
            if ((int)threadIdx.x < nc) {
                A gc = A(0);
                for (int l = 0; l < nc; ++l) gc += sg[threadIdx.x][l] * sc[l];
                c2 = sc[threadIdx.x] - gc;
            }
            // c2 = c - G c corrects for G != I but not for the rounding of c
            // itself (about u_A ||w|| per coefficient, u_A the unit roundoff
            // of the dots), which stays in the new vector: its orthogonality
            // loss is about u_A ||w|| / ||w - V c||.  Where that exceeds 100
            // times the storage rounding u_s (strong cancellation, a beta far
            // below ||A v_j||), the second coefficients are re-measured from
            // w' = w - V c, as classical Gram-Schmidt twice does
            // (k_orth_upd_dot), and the update then uses those.
            // Only where the dots are no more precise than the storage (FP64
            // storage, and the all-FP32 arithmetic): with FP32 or BF16
            // storage and FP64 dots the loss stays below the storage rounding
            // until ||w - V c|| is far under the breakdown threshold, so the
            // iteration launcher leaves the re-measuring kernel out there.
            const A ua = sizeof(A) == 8 ? A(1.1102230246251565e-16) : A(5.9604644775390625e-08);
            const bool can_remeasure = (double)ua >= st->u_s;
            const bool selective = st->reorth == 3 && st->mode != MODE_RESTART;
            // ||w - V c||^2 = ||w||^2 - 2 c.c + c.(G c) tells how much the
            // first pass cancelled.
            A sel[3] = {A(0), A(0), A(0)};
            if (can_remeasure || selective) {
                sel[0] = (int)threadIdx.x < nc ? c2 * c2 : A(0);
                sel[1] = (int)threadIdx.x < nc ? sc[threadIdx.x] * sc[threadIdx.x] : A(0);
                sel[2] = (int)threadIdx.x < nc ? sc[threadIdx.x] * (sc[threadIdx.x] - c2) : A(0);
                for (int q = 0; q < 3; ++q) sel[q] = block_sum(sel[q], shd, OWAVES);
            }
            const A w1 = fmax(A(0), wn - A(2) * sel[1] + sel[2]);
            const A lim = ua / (A(100) * (A)st->u_s);
            const bool remeasure = can_remeasure && w1 < lim * lim * wn;
            // Selective: skip the correction when it is below the rounding of
            // the stored vector, ||c2|| <= u_s ||w - V c||.  The two-pass mode
            // and restart vectors always apply it.
            bool corr = true;
            if (selective) {
                corr = sel[0] > (A)(st->u_s * st->u_s) * w1;
                if (threadIdx.x == 0) st->wnorm2 = (double)w1;
            }
            if (!remeasure && (int)threadIdx.x < nc)
                st->c2[threadIdx.x] = (double)(sc[threadIdx.x] + (corr ? c2 : A(0)));
            if (threadIdx.x == 0) {
                st->second = 1;
                st->remeasure = remeasure ? 1 : 0;
                // alpha_j = v_j . A v_j = c_j + beta_j (v_j . v_{j-1}), with
                // w = A v_j - beta_j v_{j-1}; the SpMV does not reduce it in
                // these modes.
                if (st->mode == MODE_NORMAL)
                    st->alpha[j] = (double)(sc[j] + (j > 0 ? (A)st->beta[j] * (A)gm[j * NCMAX + (j - 1)] : A(0)));
            }
        } else if (!upd_dot_active(st)) {  // one pass: the store kernel uses c
            for (int k = threadIdx.x; k < nc; k += OBLOCK) st->c2[k] = st->c[k];
            if (threadIdx.x == 0) st->second = 1;
        }
    }
}

// Partial update u = sum_k V[rows, k] coef[k] over this lane's columns,
// completed over the CS lanes of the row group.
template <int P, int NC, class A>
__device__ __forceinline__ void split_update(const typename Ch<P>::T (&ch)[Split<P, NC>::NCL], const A* coef,
                                             int cs, int lo, int nc, A (&u)[Ch<P>::R]) {
    constexpr int R = Ch<P>::R, CS = Split<P, NC>::CS, NCL = Split<P, NC>::NCL;
#pragma unroll
    for (int rr = 0; rr < R; ++rr) u[rr] = A(0);
#pragma unroll
    for (int kk = 0; kk < NCL; ++kk) {
        const int k = cs * NCL + kk;
        if (k >= lo && k < nc) {
            A v[R];
            unpack(ch[kk], v);
            const A cf = coef[k];
#pragma unroll
            for (int rr = 0; rr < R; ++rr) u[rr] += v[rr] * cf;
        }
    }
#pragma unroll
    for (int o = 1; o < CS; o <<= 1)
#pragma unroll
        for (int rr = 0; rr < R; ++rr) u[rr] += __shfl_xor(u[rr], o, 64);
}

// w' = w - V c (stored in the working precision), then c2 = V^T w' and ||w'||^2.
template <int P, int NC, class A>
__global__ __launch_bounds__(OBLOCK) void k_orth_upd_dot(State* st, const typename Tr<P>::V* __restrict__ Vb,
                                                        typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                        double* part, double* part2) {
    using CT = typename Ch<P>::T;
    constexpr int R = Ch<P>::R, CS = Split<P, NC>::CS, NCL = Split<P, NC>::NCL, GPW = 64 / CS;
    __shared__ A coef[NC];
    __shared__ A red[OWAVES][NC];
    __shared__ A shd[OWAVES];
    __shared__ A sred[OBLOCK];
    __shared__ int s_last;
    const int j = st->j;
    if (st->status != 0 || j >= st->m || !upd_dot_active(st)) return;
    const int nc = j + 1;
    if (nc > NC) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    for (int k = threadIdx.x; k < NC; k += OBLOCK) coef[k] = k < nc ? (A)st->c[k] * (A)st->scale[k] : A(0);
    __syncthreads();
    const int ln = threadIdx.x & 63, cs = ln % CS;
    constexpr int64_t RBW = (int64_t)GPW * R;
    const int64_t lane_row = (int64_t)(ln / CS) * R;
    const int64_t wave0 = (int64_t)blockIdx.x * OWAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    A acc[NCL];
#pragma unroll
    for (int kk = 0; kk < NCL; ++kk) acc[kk] = A(0);
    A nrm = A(0);
    for (int64_t base = wave0 * RBW; base < ld; base += (int64_t)gridDim.x * OWAVES * RBW) {
        const int64_t r0 = base + lane_row;
        A x[R];
        w_load(w + r0, x);
        CT ch[NCL];
#pragma unroll
        for (int kk = 0; kk < NCL; ++kk) {
            const int k = cs * NCL + kk;
            if (k < nc) ch[kk] = *(const CT*)(Vb + (int64_t)k * ld + r0);
        }
        A u[R];
        split_update<P, NC>(ch, coef, cs, 0, nc, u);
#pragma unroll
        for (int kk = 0; kk < NCL; ++kk) opaque(ch[kk]);
#pragma unroll
        for (int rr = 0; rr < R; ++rr) x[rr] -= u[rr];
        w_round_store(w + r0, x, cs == 0);
        if (cs == 0)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) nrm += x[rr] * x[rr];
#pragma unroll
        for (int kk = 0; kk < NCL; ++kk) {
            const int k = cs * NCL + kk;
            if (k < nc) {
                A v[R];
                unpack(ch[kk], v);
                A s = A(0);
#pragma unroll
                for (int rr = 0; rr < R; ++rr) s += v[rr] * x[rr];
                acc[kk] += s;
            }
        }
    }
    publish_split<NC, CS, NCL>(acc, nc, part, red);
    nrm = block_sum(nrm, shd, OWAVES);
    if (threadIdx.x == 0) st_dev(&part2[blockIdx.x], (double)nrm);
    if (last_block(&st->ticket[TK_UPD], gridDim.x, &s_last)) {
        const A wn = reduce_columns<NC>(part, part2, gridDim.x, nc, st->scale, st->c2, sred, shd);
        if (threadIdx.x == 0) {
            st->wnorm2 = (double)wn;
            st->second = 1;
        }
    }
}

// v_{j+1} = w - V c2 (c2 holds the total coefficients) stored in the basis
// precision into column j+1; beta_{j+1} = ||stored column||; breakdown check
// (beta <= tau = 100 u_w max_i(|alpha_i| + beta_i), u_w the unit roundoff of
// the working vector, starts a restart).  In the
// two-pass modes the same pass takes the dots of the stored column with the
// basis: the new row and column of the Gram matrix.
template <int P, int NC, bool GRAM, class A>
__global__ __launch_bounds__(OBLOCK) void k_orth_upd_store(State* st, typename Tr<P>::V* __restrict__ Vb,
                                                          const typename Tr<P>::W* __restrict__ w, int64_t ld,
                                                          double* part, double* part2, double* gm) {
    using CT = typename Ch<P>::T;
    constexpr int R = Ch<P>::R, CS = Split<P, NC>::CS, NCL = Split<P, NC>::NCL, GPW = 64 / CS;
    __shared__ A coef[NC];
    __shared__ A red[OWAVES][NC];
    __shared__ double gcol[NC];
    __shared__ A sha[OWAVES];
    __shared__ double shd[OWAVES];
    __shared__ A sred[OBLOCK];
    __shared__ int s_last, s_accept;
    // The coefficients do not depend on the step index: their loads go out
    // with it.
    double c2k = 0.0, sk = 0.0;
    if ((int)threadIdx.x < NC) {
        c2k = st->c2[threadIdx.x];
        sk = st->scale[threadIdx.x];
    }
    const int j = st->j;
    if (st->status != 0 || j >= st->m) return;
    const int nc = j + 1;
    if (nc > NC) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->status = -1;
        return;
    }
    // The Gram variant runs in the two-pass modes, where every column takes
    // part in the update.
    const bool second = GRAM || st->second != 0;
    constexpr bool gram = GRAM;
    const int lo = (!GRAM && st->reorth == 0 && st->mode != MODE_RESTART) ? j : 0;
    if ((int)threadIdx.x < NC) {
        const int k = threadIdx.x;
        coef[k] = (second && k >= lo && k < nc) ? (A)c2k * (A)sk : A(0);
    }
    __syncthreads();
    const int ln = threadIdx.x & 63, cs = ln % CS;
    constexpr int64_t RBW = (int64_t)GPW * R;
    const int64_t lane_row = (int64_t)(ln / CS) * R;
    const int64_t wave0 = (int64_t)blockIdx.x * OWAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto* out = Vb + (int64_t)(j + 1) * ld;
    A nrm = A(0);
    A acc[NCL];
#pragma unroll
    for (int kk = 0; kk < NCL; ++kk) acc[kk] = A(0);
    for (int64_t base = wave0 * RBW; base < ld; base += (int64_t)gridDim.x * OWAVES * RBW) {
        const int64_t r0 = base + lane_row;
        A x[R];
        w_load(w + r0, x);
        if (second) {
            CT ch[NCL];
#pragma unroll
            for (int kk = 0; kk < NCL; ++kk) {
                const int k = cs * NCL + kk;
                if (k >= lo && k < nc) ch[kk] = *(const CT*)(Vb + (int64_t)k * ld + r0);
            }
            A u[R];
            split_update<P, NC>(ch, coef, cs, lo, nc, u);
#pragma unroll
            for (int kk = 0; kk < NCL; ++kk) opaque(ch[kk]);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) x[rr] -= u[rr];
            v_round_store(out + r0, x, cs == 0);
            if (gram)
#pragma unroll
                for (int kk = 0; kk < NCL; ++kk) {
                    const int k = cs * NCL + kk;
                    if (k < nc) {
                        A v[R];
                        unpack(ch[kk], v);
                        A s = A(0);
#pragma unroll
                        for (int rr = 0; rr < R; ++rr) s += v[rr] * x[rr];
                        acc[kk] += s;
                    }
                }
        } else {
            v_round_store(out + r0, x, cs == 0);
        }
        if (cs == 0)
#pragma unroll
            for (int rr = 0; rr < R; ++rr) nrm += x[rr] * x[rr];
    }
    if (gram) publish_split<NC, CS, NCL>(acc, nc, part, red);
    nrm = block_sum(nrm, sha, OWAVES);
    if (threadIdx.x == 0) st_dev(&part2[blockIdx.x], (double)nrm);
    if (last_block(&st->ticket[TK_STORE], gridDim.x, &s_last)) {
        const A tot = gram ? reduce_columns<NC>(part, part2, gridDim.x, nc, st->scale, gcol, sred, sha)
                           : (A)ordered_sum_dev(part2, gridDim.x, shd);
        if (threadIdx.x == 0) {
            const A b = sqrt(tot);
            int accept = 0;
            if (!isfinite(b)) {
                st->status = -7;               // LZ_ERR_NONFINITE
                st->j = st->m;
            } else if (st->mode == MODE_NORMAL) {
                const double t = fabs(st->alpha[j]) + st->beta[j];
                if (t > st->tnorm) st->tnorm = t;
                const double tau = 100.0 * st->u_w * st->tnorm;
                if (!(b > tau) && j + 1 < st->m) {
                    // Breakdown: the Krylov space is invariant.  T gets a zero
                    // coupling and the next iteration draws a restart vector.
                    st->mode = MODE_RESTART;
                    st->restarts += 1;
                    st->beta[j + 1] = 0.0;
                } else {
                    st->beta[j + 1] = (double)b;
                    st->scale[j + 1] = b > A(0) ? (double)(A(1) / b) : 0.0;
                    st->j = j + 1;
                    accept = 1;
                }
            } else {
                if (!(b > 0.0)) {
                    st->status = -8;           // LZ_ERR_BREAKDOWN
                    st->j = st->m;
                } else {
                    st->scale[j + 1] = (double)(A(1) / b);
                    st->beta[j + 1] = 0.0;
                    st->mode = MODE_NORMAL;
                    st->j = j + 1;
                    accept = 1;
                }
            }
            s_accept = accept;
        }
        __syncthreads();
        if (gram && s_accept) {
            // Gram entries of the unit stored vectors: column j+1 against 0..j
            // (gcol already carries scale_k) and its own squared norm.
            const A sn = (A)st->scale[j + 1];
            for (int k = threadIdx.x; k < nc; k += OBLOCK) {
                const double g = (double)((A)gcol[k] * sn);
                gm[k * NCMAX + (j + 1)] = g;
                gm[(j + 1) * NCMAX + k] = g;
            }
            if (threadIdx.x == 0) gm[(j + 1) * NCMAX + (j + 1)] = (double)(tot * sn * sn);
        }
    }
}

// ---------------------------------------------------------------- launchers
static inline int nc_bucket(int ncols) { return ((ncols + 7) / 8) * 8; }

template <int P, class A>
static hipError_t iteration_pa(const Plan& p, const Bufs& b, const Csr& a, int ncols, int reorth, hipStream_t s,
                               hipEvent_t* ev) {
    using VT = typename Tr<P>::V;
    using WT = typename Tr<P>::W;
    VT* V = (VT*)b.V;
    WT* w = (WT*)b.w;
    // The final reductions of the orthogonalisation kernels read at most
    // OGRID partial rows.
    if (p.g_orth < 1 || p.g_orth > OGRID) return hipErrorInvalidValue;
    if (ev) (void)hipEventRecord(ev[0], s);
    const hipError_t es = launch_spmv_step(p, b, a, s);
    if (es != hipSuccess) return es;
    if (ev) (void)hipEventRecord(ev[1], s);
    const int nb = nc_bucket(ncols);
    // The two-pass modes re-measure their second coefficients only where the
    // dots are no more precise than the storage (see k_orth_dot).
    const bool remeasure_possible = P == 0 || sizeof(A) == 4;
#define LZ_ORTH_CASE(NCV)                                                                                  \
    case NCV:                                                                                              \
        hipLaunchKernelGGL((k_orth_dot<P, NCV, A>), dim3(p.g_orth), dim3(OBLOCK), 0, s, b.st, V, w, p.ld,      \
                           b.part, b.part2, b.gm);                                                         \
        if (reorth < 2 || remeasure_possible)                                                              \
            hipLaunchKernelGGL((k_orth_upd_dot<P, NCV, A>), dim3(p.g_orth), dim3(OBLOCK), 0, s, b.st, V, w,    \
                               p.ld, b.part, b.part2);                                                     \
        if (reorth >= 2)                                                                                   \
            hipLaunchKernelGGL((k_orth_upd_store<P, NCV, true, A>), dim3(p.g_orth), dim3(OBLOCK), 0, s, b.st, V, \
                               w, p.ld, b.part, b.part2, b.gm);                                            \
        else                                                                                               \
            hipLaunchKernelGGL((k_orth_upd_store<P, NCV, false, A>), dim3(p.g_orth), dim3(OBLOCK), 0, s, b.st,  \
                               V, w, p.ld, b.part, b.part2, b.gm);                                         \
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
        default:
            return hipErrorInvalidValue;
    }
#undef LZ_ORTH_CASE
    return hipGetLastError();
}

hipError_t launch_iteration(const Plan& p, const Bufs& b, const Csr& a, int ncols, int reorth, hipStream_t s,
                            hipEvent_t* ev) {
    switch (p.prec) {
        case 0: return iteration_pa<0, double>(p, b, a, ncols, reorth, s, ev);
        case 1:
            return p.fff ? iteration_pa<1, float>(p, b, a, ncols, reorth, s, ev)
                         : iteration_pa<1, double>(p, b, a, ncols, reorth, s, ev);
        case 2: return iteration_pa<2, double>(p, b, a, ncols, reorth, s, ev);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(const Plan& p, const Bufs& b, hipStream_t s) {
    switch (p.prec) {
        case 0:
            hipLaunchKernelGGL(k_init<0>, dim3(p.g_dense), dim3(BLOCK), 0, s, b.st, (double*)b.V, (double*)b.w, p.n,
                               p.ld, b.part2, b.gm);
            break;
        case 1:
            hipLaunchKernelGGL(k_init<1>, dim3(p.g_dense), dim3(BLOCK), 0, s, b.st, (float*)b.V, (float*)b.w, p.n,
                               p.ld, b.part2, b.gm);
            break;
        case 2:
            hipLaunchKernelGGL(k_init<2>, dim3(p.g_dense), dim3(BLOCK), 0, s, b.st, (uint16_t*)b.V, (float*)b.w,
                               p.n, p.ld, b.part2, b.gm);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lz
