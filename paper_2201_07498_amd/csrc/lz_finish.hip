// gfx950 kernels after the Lanczos loop (Sec. III, second phase): Jacobi on
// the tridiagonal T, Top-K selection, Ritz vectors, and the accuracy report
// of Sec. IV-D (residuals, orthogonality of the basis and of the Ritz
// vectors, mean pairwise angle).
#include <algorithm>
#include <cmath>

#include "lz_ooc.h"
#include "lz_spmv.h"

namespace lz {

constexpr int JMAX_SWEEPS = 60;
constexpr int JBLOCK = 1024;      // Jacobi workgroup: one round is a single parallel step

// ---------------------------------------------------------------- Jacobi
// Parallel cyclic Jacobi in LDS.  Each round applies me/2 disjoint
// rotations chosen by the round-robin tournament ordering (me = m rounded up
// to even; an odd m gets a zero dummy row and column that is never
// rotated); me-1 rounds make a sweep.  Rotation (Rutishauser):
// zeta = (t_qq - t_pp)/(2 t_pq), t = sgn(zeta)/(|zeta| + sqrt(1+zeta^2)),
// c = 1/sqrt(1+t^2), s = t c.  A rotation is skipped when |t_pq| is
// negligible (<= eps sqrt|t_pp t_qq| or <= eps^2 ||T||_F); the method stops
// at a sweep without rotations (counted, not run).
//
// Disjoint rotations commute, so a round is one parallel step: T' = J^T T J
// is updated as independent 2x2 blocks (rows of pair a, columns of pair b),
// upper blocks computed and mirrored so T stays exactly symmetric, and S' = S J.
__device__ void jacobi_core(int m, double (*T)[MMAX + 1], double (*S)[MMAX + 1], double fro, int* sweeps_out,
                            int* rot_flag) {
    __shared__ double rc[MMAX / 2], rs[MMAX / 2];
    __shared__ int rp_[MMAX / 2], rq_[MMAX / 2], rr_[MMAX / 2];
    __shared__ uint8_t pair_p[MMAX - 1][MMAX / 2], pair_q[MMAX - 1][MMAX / 2];
    __shared__ uint8_t blk_a[MMAX / 2 * (MMAX / 2 + 1) / 2], blk_b[MMAX / 2 * (MMAX / 2 + 1) / 2];
    const double eps = 1.1102230246251565e-16;
    const int me = (m + 1) & ~1;
    const int half = me / 2;
    const int nt = blockDim.x;
    const int nblk = half * (half + 1) / 2;
    // Threads for the T blocks (whole wavefronts, at most half the
    // workgroup).  Splitting pays while the remaining threads need at most two
    // S items each (measured: m = 48 faster by 10%, m = 64 slower by 14%);
    // otherwise 0, and every thread takes both updates in turn.
    const int split_t = (min(nblk, nt / 2) + 63) & ~63;
    const int split = (split_t < nt && me * half <= 2 * (nt - split_t)) ? split_t : 0;
    // Tournament pairs of every round and the upper 2x2 block list, once.
    for (int idx = threadIdx.x; idx < (me - 1) * half; idx += nt) {
        const int round = idx / half, i = idx % half;
        auto pos = [&](int k) { return k == 0 ? 0 : 1 + ((k - 1 + round) % (me - 1)); };
        const int p = pos(i), q = pos(me - 1 - i);
        pair_p[round][i] = (uint8_t)min(p, q);
        pair_q[round][i] = (uint8_t)max(p, q);
    }
    for (int a = threadIdx.x; a < half; a += nt) {
        const int first = a * half - a * (a - 1) / 2;      // blocks (a', b) with a' < a come first
        for (int b = a; b < half; ++b) {
            blk_a[first + b - a] = (uint8_t)a;
            blk_b[first + b - a] = (uint8_t)b;
        }
    }
    __syncthreads();
    int sweeps = -1;
    for (int sweep = 1; sweep <= JMAX_SWEEPS; ++sweep) {
        // A sweep rotates nothing exactly when every pair already passes the
        // skip test at its start (T does not change within such a sweep), so
        // that sweep is detected here instead of being run.
        if (threadIdx.x == 0) *rot_flag = 0;
        __syncthreads();
        for (int idx = threadIdx.x; idx < m * m; idx += nt) {
            const int p = idx / m, q = idx % m;
            if (p < q) {
                const double apq = T[p][q];
                if (!(fabs(apq) <= eps * sqrt(fabs(T[p][p] * T[q][q])) || fabs(apq) <= eps * eps * fro))
                    *rot_flag = 1;
            }
        }
        __syncthreads();
        const int pending = *rot_flag;
        __syncthreads();
        if (!pending) {
            sweeps = sweep;
            break;
        }
        if (threadIdx.x == 0) *rot_flag = 0;
        __syncthreads();
        for (int round = 0; round < me - 1; ++round) {
            for (int i = threadIdx.x; i < half; i += nt) {
                const int p = pair_p[round][i], q = pair_q[round][i];
                double c = 1.0, s = 0.0;
                int rot = 0;
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
                    rot = 1;
                    *rot_flag = 1;
                }
                rc[i] = c;
                rs[i] = s;
                rp_[i] = p;
                rq_[i] = q;
                rr_[i] = rot;
            }
            __syncthreads();
            // Upper 2x2 blocks (a <= b) of J^T T J, mirrored to the lower half.
            auto t_block = [&](int idx) {
                const int a = blk_a[idx], b = blk_b[idx];
                if (!rr_[a] && !rr_[b]) return;
                const int pa = rp_[a], qa = rq_[a], pb = rp_[b], qb = rq_[b];
                const double ca = rc[a], sa = rs[a], cb = rc[b], sb = rs[b];
                const double t00 = T[pa][pb], t01 = T[pa][qb], t10 = T[qa][pb], t11 = T[qa][qb];
                const double u00 = ca * t00 - sa * t10, u01 = ca * t01 - sa * t11;
                const double u10 = sa * t00 + ca * t10, u11 = sa * t01 + ca * t11;
                double v00 = cb * u00 - sb * u01, v01 = sb * u00 + cb * u01;
                double v10 = cb * u10 - sb * u11, v11 = sb * u10 + cb * u11;
                if (a == b) {
                    v01 = 0.0;                  // the annihilated entry
                    v10 = 0.0;
                }
                T[pa][pb] = v00;
                T[pa][qb] = v01;
                T[qa][pb] = v10;
                T[qa][qb] = v11;
                if (a != b) {
                    T[pb][pa] = v00;
                    T[qb][pa] = v01;
                    T[pb][qa] = v10;
                    T[qb][qa] = v11;
                }
            };
            // S' = S J, row r of the columns of pair b.
            auto s_item = [&](int idx) {
                const int r = idx / half, b = idx - r * half;
                if (!rr_[b]) return;
                const int pb = rp_[b], qb = rq_[b];
                const double sp = S[r][pb], sq = S[r][qb];
                S[r][pb] = rc[b] * sp - rs[b] * sq;
                S[r][qb] = rs[b] * sp + rc[b] * sq;
            };
            // The two updates are independent: with enough wavefronts, the
            // first `split` threads take the T blocks and the others the S
            // rows, so the two run side by side.
            if (split > 0) {
                if ((int)threadIdx.x < split)
                    for (int idx = threadIdx.x; idx < nblk; idx += split) t_block(idx);
                else
                    for (int idx = threadIdx.x - split; idx < me * half; idx += nt - split) s_item(idx);
            } else {
                for (int idx = threadIdx.x; idx < nblk; idx += nt) t_block(idx);
                for (int idx = threadIdx.x; idx < me * half; idx += nt) s_item(idx);
            }
            __syncthreads();
        }
    }
    *sweeps_out = sweeps;
}

// T (me x me, zero-padded) from a diagonal and an off-diagonal array.
__device__ void jacobi_load_tridiag(int m, const double* diag, const double* off, int off_shift,
                                    double (*T)[MMAX + 1], double (*S)[MMAX + 1], double* sh, double* fro) {
    const int me = (m + 1) & ~1;
    double f = 0.0;
    for (int idx = threadIdx.x; idx < me * me; idx += blockDim.x) {
        const int r = idx / me, c = idx % me;
        double t = 0.0;
        if (r < m && c < m) {
            if (r == c) t = diag[r];
            else if (c == r + 1) t = off[r + off_shift];
            else if (r == c + 1) t = off[c + off_shift];
        }
        T[r][c] = t;
        S[r][c] = r == c ? 1.0 : 0.0;
        f += t * t;
    }
    *fro = sqrt(block_sum(f, sh, blockDim.x / 64));
    __syncthreads();
}

// T from alpha_1..alpha_m and beta_2..beta_m, Jacobi, Top-K selection by
// modulus (ties: larger value, then lower index); writes the eigenvalues.
// With `strict` (stream-ordered calls, whose iteration budget is fixed when
// they are enqueued), a solve that completed fewer than m steps because more
// breakdowns occurred than the budget absorbs ends with LZ_ERR_RESTART_BUDGET.
__global__ __launch_bounds__(JBLOCK) void k_jacobi_select(State* st, double* out_vals, int strict) {
    __shared__ double T[MMAX][MMAX + 1];
    __shared__ double S[MMAX][MMAX + 1];
    __shared__ double shd[JBLOCK / 64];
    __shared__ int rot_flag, sweeps;
    if (st->status != 0) return;
    if (strict && st->j < st->m) {
        if (threadIdx.x == 0) st->status = -9;     // LZ_ERR_RESTART_BUDGET
        return;
    }
    const int m = min(st->j, st->m);
    const int K = st->K;
    if (m < K) {
        if (threadIdx.x == 0) st->status = -8;
        return;
    }
    double fro;
    jacobi_load_tridiag(m, st->alpha, st->beta, 1, T, S, shd, &fro);
    jacobi_core(m, T, S, fro, &sweeps, &rot_flag);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) st->theta[i] = T[i][i];
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) st->S[(idx / m) * MMAX + idx % m] = S[idx / m][idx % m];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double ti = T[i][i];
        int rank = 0;
        for (int k = 0; k < m; ++k) {
            const double tk = T[k][k];
            rank += fabs(tk) > fabs(ti) || (fabs(tk) == fabs(ti) && (tk > ti || (tk == ti && k < i)));
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
__global__ __launch_bounds__(JBLOCK) void k_jacobi_only(const double* alpha, const double* offd, int m, State* st) {
    __shared__ double T[MMAX][MMAX + 1];
    __shared__ double S[MMAX][MMAX + 1];
    __shared__ double shd[JBLOCK / 64];
    __shared__ int rot_flag, sweeps;
    double fro;
    jacobi_load_tridiag(m, alpha, offd, 0, T, S, shd, &fro);
    jacobi_core(m, T, S, fro, &sweeps, &rot_flag);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) st->theta[i] = T[i][i];
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) st->S[(idx / m) * MMAX + idx % m] = S[idx / m][idx % m];
    if (threadIdx.x == 0) {
        st->sweeps = sweeps;
        st->status = sweeps < 0 ? -6 : 0;
    }
}

// ------------------------------------------------------------ Ritz vectors
// Y[r][k] = sum_i scale_i V[r,i] S[i, sel_k]  (eigenvectors of the matrix are
// the Lanczos basis times those of T).  Y is row-major n x K (a K-wide row
// per matrix row, the layout the residual SpMM gathers), not normalised.
template <int P, int KB>
__global__ __launch_bounds__(BLOCK) void k_ritz(const State* st, const typename Tr<P>::V* __restrict__ Vb, int64_t n,
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

// Per Ritz column k: norm and the entry of largest modulus (lowest original
// row on ties) -> ysc[k] = sign(that entry) / norm.  Lane k of each group of
// KB2 lanes owns column k.  NOROW marks "no row yet" (exact as a double and
// as an int64).
constexpr int64_t NOROW = int64_t(1) << 62;
__global__ __launch_bounds__(BLOCK) void k_colstats(State* st, const double* __restrict__ Y, int64_t n, int KB2,
                                                    double* part) {
    __shared__ double s_n[BLOCK], s_a[BLOCK], s_v[BLOCK];
    __shared__ int64_t s_i[BLOCK];
    __shared__ int s_last;
    if (st->status != 0) return;
    const int K = st->K, G = gridDim.x;
    const int groups = BLOCK / KB2, g = threadIdx.x / KB2, k = threadIdx.x % KB2;
    double nrm = 0.0, best = -1.0, bval = 0.0;
    int64_t bidx = NOROW;
    const int32_t* perm = st->perm;
    auto visit = [&](int64_t r, double v) {
        nrm += v * v;
        const double a = fabs(v);
        const int64_t ro = perm ? perm[r] : r;
        if (a > best || (a == best && ro < bidx)) { best = a; bval = v; bidx = ro; }
    };
    if (k < K) {
        const int64_t S = (int64_t)G * groups;
        int64_t r = (int64_t)blockIdx.x * groups + g;
        for (; r + 3 * S < n; r += 4 * S) {       // four rows in flight
            const double v0 = Y[r * K + k], v1 = Y[(r + S) * K + k], v2 = Y[(r + 2 * S) * K + k],
                         v3 = Y[(r + 3 * S) * K + k];
            visit(r, v0);
            visit(r + S, v1);
            visit(r + 2 * S, v2);
            visit(r + 3 * S, v3);
        }
        for (; r < n; r += S) visit(r, Y[r * K + k]);
    }
    s_n[threadIdx.x] = nrm; s_a[threadIdx.x] = best; s_v[threadIdx.x] = bval; s_i[threadIdx.x] = bidx;
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double tn = 0.0, ta = -1.0, tv = 0.0;
        int64_t ti = NOROW;
        for (int gg = 0; gg < groups; ++gg) {
            const int t = gg * KB2 + threadIdx.x;
            tn += s_n[t];
            if (s_a[t] > ta || (s_a[t] == ta && s_i[t] < ti)) { ta = s_a[t]; tv = s_v[t]; ti = s_i[t]; }
        }
        double* pb = part + ((int64_t)blockIdx.x * 64 + threadIdx.x) * 4;
        st_dev(pb + 0, tn);
        st_dev(pb + 1, ta);
        st_dev(pb + 2, tv);
        st_dev(pb + 3, (double)ti);
    }
    if (last_block(&st->ticket[TK_RITZ], (uint32_t)G, &s_last)) {
        // Thread (g, k) folds workgroups g, g + groups, ... of column k (four
        // loads in flight), then the groups are folded in order.
        double tn = 0.0, ta = -1.0, tv = 0.0, ti = (double)NOROW;
        auto fold = [&](const double* pb) {
            const double nn = ld_dev(pb), a = ld_dev(pb + 1), v = ld_dev(pb + 2), i = ld_dev(pb + 3);
            tn += nn;
            if (a > ta || (a == ta && i < ti)) { ta = a; tv = v; ti = i; }
        };
        if (k < K) {
            int b = g;
            for (; b + 3 * groups < G; b += 4 * groups) {
                const double* p0 = part + ((int64_t)b * 64 + k) * 4;
                const double* p1 = part + ((int64_t)(b + groups) * 64 + k) * 4;
                const double* p2 = part + ((int64_t)(b + 2 * groups) * 64 + k) * 4;
                const double* p3 = part + ((int64_t)(b + 3 * groups) * 64 + k) * 4;
                fold(p0);
                fold(p1);
                fold(p2);
                fold(p3);
            }
            for (; b < G; b += groups) fold(part + ((int64_t)b * 64 + k) * 4);
        }
        s_n[threadIdx.x] = tn; s_a[threadIdx.x] = ta; s_v[threadIdx.x] = tv; s_i[threadIdx.x] = (int64_t)ti;
        __syncthreads();
        if ((int)threadIdx.x < K) {
            double n2 = 0.0, a2 = -1.0, v2 = 0.0;
            int64_t i2 = NOROW;
            for (int gg = 0; gg < groups; ++gg) {
                const int t = gg * KB2 + threadIdx.x;
                n2 += s_n[t];
                if (s_a[t] > a2 || (s_a[t] == a2 && s_i[t] < i2)) { a2 = s_a[t]; v2 = s_v[t]; i2 = s_i[t]; }
            }
            st->ysc[threadIdx.x] = (v2 < 0.0 ? -1.0 : 1.0) / sqrt(n2);
        }
    }
}

// Residual check (Sec. IV-D) in FP64 for all K Ritz pairs at once.
// First Z = A Y (stored matrix values upcast exactly) over the SpMV tiles:
// each wavefront stages its tile's col/val in LDS (values in the storage
// precision, upcast when used); lane k of a group of KB2
// lanes owns pair k and gathers K-wide rows of Y.  Rows are spread over the
// 64/KB2 groups; a row longer than LONGZ, and a split row's piece, is shared
// by all groups.  Split rows are finished by their last piece as in the
// SpMV, the pieces added in tile order.
constexpr int LONGZ = 32;

// sum over p = p0, p0+step, ... < e of sval[p] * Y[scol[p]][k].  Eight
// gathers per lane are issued together, those past the end clamped to the
// batch's first entry and discarded, so a row of up to eight entries costs
// one round of requests; fixed association order.
template <class VT>
__device__ __forceinline__ double gather_dot(const int* scol, const VT* sval, int p0, int e, int step,
                                             const double* __restrict__ Y, int K, int k) {
    double z[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int p = p0; p < e; p += 8 * step) {
        double y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int q = p + i * step < e ? p + i * step : p;
            y[i] = Y[(int64_t)scol[q] * K + k];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int q = p + i * step;
            z[i] += q < e ? to_d(sval[q]) * y[i] : 0.0;
        }
    }
    return ((z[0] + z[1]) + (z[2] + z[3])) + ((z[4] + z[5]) + (z[6] + z[7]));
}

// Adds the groups' values (lanes that differ in the group bits), fixed order.
__device__ __forceinline__ double group_sum(double v, int KB2) {
    for (int o = KB2; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The matrix arrays come in as kernel arguments (the caller's CSR and the
// relabelled copy), so their loads are global loads, as in the step SpMV.
template <int P>
__global__ __launch_bounds__(BLOCK) void k_spmm(State* st, const double* __restrict__ Y, double* __restrict__ Z,
                                                int64_t n, int64_t nnz, int64_t n_tiles, const int32_t* __restrict__ ob,
                                                uint32_t* tk, double* head, double* tail, int KB2,
                                                const int64_t* rp_a, const int32_t* col_a, const void* val_a,
                                                const int64_t* rp_b, const int32_t* col_b, const void* val_b,
                                                int64_t tb, int64_t te) {
    using VT = typename Tr<P>::V;
    __shared__ int scol_all[WAVES][TILE];
    __shared__ VT sval_all[WAVES][TILE];
    if (st->status != 0) return;
    const bool rl = st->reordered != 0;
    const int packing = rl ? st->packed : PACK_NONE;
    const int64_t* rp = rl ? rp_b : rp_a;
    const int32_t* col = rl ? col_b : col_a;
    const VT* val = (const VT*)(rl ? val_b : val_a);
    const int K = st->K;
    const int lane = threadIdx.x & 63;
    const int G = 64 / KB2, g = lane / KB2, k = lane % KB2;
    const bool act = k < K;
    int* scol = scol_all[threadIdx.x >> 6];
    VT* sval = sval_all[threadIdx.x >> 6];
    // Pieces of split row r (tail pieces in t1..t2-1, head piece in t2),
    // added group-strided in tile order; the whole row sum in every group.
    auto split_total_k = [&](int64_t t1, int64_t t2) {
        double z = 0.0;
        if (act)
            for (int64_t i = t1 + g; i < t2; i += G) z += ld_dev(&tail[i * KB2 + k]);
        z = group_sum(z, KB2);
        return act ? z + ld_dev(&head[t2 * KB2 + k]) : 0.0;
    };
    // Rows of tile t from its entries in row order, scol/sval[0..cnt).
    auto tile_body = [&](int64_t t, const int* scol, const VT* sval) {
        const int64_t r_lo = ob[t], r_hi = ob[t + 1];
        const int64_t t0 = t * TILE - r_lo;
        const int cnt = (int)(min<int64_t>((t + 1) * TILE, nnz + n) - r_hi - t0);
        const bool split_head = r_lo < r_hi && rp[r_lo] < t0;
        double head_z = 0.0;
        for (int64_t base = r_lo; base < r_hi; base += G) {
            const int64_t r = base + g;
            const bool valid = r < r_hi;
            int b = 0, e = 0;
            if (valid) {
                b = (int)(max(rp[r], t0) - t0);
                e = (int)(rp[r + 1] - t0);
            }
            const bool islong = valid && e - b > LONGZ;
            double z = (valid && !islong && act) ? gather_dot(scol, sval, b, e, 1, Y, K, k) : 0.0;
            uint64_t mask = __ballot(islong && k == 0);
            while (mask) {
                const int L = __builtin_ctzll(mask);
                mask &= mask - 1;
                const int bL = __shfl(b, L, 64), eL = __shfl(e, L, 64);
                double zz = act ? gather_dot(scol, sval, bL + g, eL, G, Y, K, k) : 0.0;
                zz = group_sum(zz, KB2);
                if (g == L / KB2) z = zz;
            }
            if (valid && act) {
                if (split_head && r == r_lo)
                    head_z = z;
                else
                    Z[r * K + k] = z;
            }
        }
        if (split_head) {
            if (g == 0 && act) st_dev(&head[t * KB2 + k], head_z);
            const int64_t t1 = item_tile(rp[r_lo] + r_lo, n_tiles);
            if (last_wave(&tk[t], (uint32_t)(t - t1 + 1))) {
                const double z = split_total_k(t1, t);
                if (g == 0 && act) Z[r_lo * K + k] = z;
            }
        }
        if (r_hi < n) {
            const int64_t rb = rp[r_hi];
            if (rb < t0 + cnt) {
                double zz = act ? gather_dot(scol, sval, (int)(max(rb, t0) - t0) + g, cnt, G, Y, K, k) : 0.0;
                zz = group_sum(zz, KB2);
                if (g == 0 && act) st_dev(&tail[t * KB2 + k], zz);
                const int64_t t1 = item_tile(rb + r_hi, n_tiles), t2 = row_owner(rp, r_hi, n_tiles);
                if (last_wave(&tk[t2], (uint32_t)(t2 - t1 + 1))) {
                    const double z = split_total_k(t1, t2);
                    if (g == 0 && act) Z[r_hi * K + k] = z;
                }
            }
        }
    };
    if (packing == PACK_GROUP) {
        // Group-sorted storage: the workgroup puts a group's entries back in
        // row order in its LDS, then each wavefront takes its tile.
        static_assert(WAVES == GROUP_TILES, "one wavefront per tile of a group");
        int* gcol = &scol_all[0][0];
        VT* gval = &sval_all[0][0];
        const int w = threadIdx.x >> 6;
        const int64_t n_groups = (n_tiles + GROUP_TILES - 1) / GROUP_TILES;
        const int64_t xcd = blockIdx.x & 7, nb8 = gridDim.x >> 3;
        const int64_t lo = n_groups * xcd / 8, hi = n_groups * (xcd + 1) / 8;
        for (int64_t gi = lo + (blockIdx.x >> 3); gi < hi; gi += nb8) {
            const int64_t tg = gi * GROUP_TILES, tend = min<int64_t>(tg + GROUP_TILES, n_tiles);
            const int64_t g0 = tg * TILE - ob[tg];
            const int64_t gend = tend >= n_tiles ? nnz : tend * TILE - ob[tend];
            for (int64_t i = threadIdx.x; i < gend - g0; i += BLOCK) {
                const uint32_t cw = (uint32_t)col[g0 + i];
                const int sl = (int)(cw & GROUP_SLOTMASK);
                gcol[sl] = (int)(cw >> GROUP_SLOTBITS);
                gval[sl] = val[g0 + i];
            }
            __syncthreads();
            const int64_t t = tg + w;
            if (t < n_tiles) {
                const int off = (int)(t * TILE - ob[t] - g0);
                tile_body(t, gcol + off, gval + off);
            }
            __syncthreads();
        }
        return;
    }
    const TileRange tr = wave_tiles(tb, te);
    for (int64_t t = tr.first; t < tr.end; t += tr.stride) {
        const int64_t r_lo = ob[t], r_hi = ob[t + 1];
        const int64_t t0 = t * TILE - r_lo;
        const int cnt = (int)(min<int64_t>((t + 1) * TILE, nnz + n) - r_hi - t0);
        // A tile-sorted tile goes back to row order in LDS.
        for (int i = lane; i < cnt; i += 64) {
            const uint32_t cw = (uint32_t)col[t0 + i];
            const int sl = packing == PACK_TILE ? (int)(cw & PACK_SLOTMASK) : i;
            scol[sl] = packing == PACK_TILE ? (int)(cw >> PACK_SLOTBITS) : (int)cw;
            sval[sl] = val[t0 + i];
        }
        wave_sync();
        tile_body(t, scol, sval);
        wave_sync();
    }
}

// Residuals ||A y_k - theta_k y_k|| = ||ysc_k Z[:,k] - theta_k ysc_k Y[:,k]||
// (Sec. IV-D), streaming Y and Z in the solve's row order; thread (g, k)
// sums rows g, g + groups, ... of pair k (four rows in flight), workgroup
// partials are added in a fixed order by the last workgroup.
__global__ __launch_bounds__(BLOCK) void k_resid(State* st, const double* __restrict__ Y,
                                                 const double* __restrict__ Z, int64_t n, int KB2, double* part) {
    __shared__ double shz[BLOCK];
    __shared__ int s_last;
    if (st->status != 0) return;
    const int K = st->K;
    const int tid = threadIdx.x, groups = BLOCK / KB2, g = tid / KB2, k = tid % KB2;
    const bool act = k < K;
    const double ysc = act ? st->ysc[k] : 0.0;
    const double th = act ? st->theta[st->sel[k]] : 0.0;
    double racc = 0.0;
    if (act) {
        auto term = [&](int64_t r) {
            const double y = ysc * Y[r * K + k];
            const double d = ysc * Z[r * K + k] - th * y;
            return d * d;
        };
        const int64_t S = (int64_t)gridDim.x * groups;
        int64_t r = (int64_t)blockIdx.x * groups + g;
        for (; r + 3 * S < n; r += 4 * S) {
            const double d0 = term(r), d1 = term(r + S), d2 = term(r + 2 * S), d3 = term(r + 3 * S);
            racc += d0;
            racc += d1;
            racc += d2;
            racc += d3;
        }
        for (; r < n; r += S) racc += term(r);
    }
    shz[tid] = racc;
    __syncthreads();
    if (tid < KB2) {
        double sum = 0.0;
        for (int gg = 0; gg < groups; ++gg) sum += shz[gg * KB2 + tid];
        st_dev(&part[(int64_t)blockIdx.x * 64 + tid], sum);
    }
    if (last_block(&st->ticket[TK_RESID], gridDim.x, &s_last)) {
        // Thread (g, k) adds workgroups g, g + groups, ... of column k; the
        // group sums are then added in group order.
        __syncthreads();
        shz[tid] = act ? strided_sum_dev(part + k, 64, g, groups, gridDim.x) : 0.0;
        __syncthreads();
        if (tid < K) {
            double sum = 0.0;
            for (int gg = 0; gg < groups; ++gg) sum += shz[gg * KB2 + tid];
            const double a2 = sqrt(sum);
            const double tl = st->theta[st->sel[tid]];
            st->abs_resid[tid] = a2;
            st->resid[tid] = tl != 0.0 ? a2 / fabs(tl) : a2;
        }
    }
}

// Unit Ritz vectors y_k = ysc_k Y[:,k] into the caller's column-major output
// in original row order: a 64-row block is gathered row-wise (through the
// original-to-solve row map when the matrix was relabelled) and written
// column-wise through LDS.
__global__ __launch_bounds__(BLOCK) void k_out(const State* st, const double* __restrict__ Y, int64_t n, int KB2,
                                               double* __restrict__ out) {
    __shared__ double ys[64][65];
    if (st->status != 0) return;
    const int K = st->K;
    const int tid = threadIdx.x, k = tid % KB2;
    const bool act = k < K;
    const double ysc = act ? st->ysc[k] : 0.0;
    const int32_t* iperm = st->iperm;
    for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < n; r0 += (int64_t)gridDim.x * 64) {
        for (int idx = tid; idx < 64 * KB2; idx += BLOCK) {
            const int row = idx / KB2;
            const int64_t r = r0 + row;
            if (r < n && act) {
                const int64_t i = iperm ? iperm[r] : r;
                ys[row][k] = ysc * Y[i * K + k];
            }
        }
        __syncthreads();
        for (int idx = tid; idx < 64 * K; idx += BLOCK) {
            const int kk = idx / 64, row = idx % 64;
            const int64_t r = r0 + row;
            if (r < n) out[(int64_t)kk * n + r] = ys[row][kk];
        }
        __syncthreads();
    }
}

// -------------------------------------------------------- orthogonality
// Gram matrix G = X^T X of c <= 64 columns (column k scaled by scale[k]) on
// the FP64 matrix cores.  A workgroup stages panels of 64 rows x c columns in
// LDS (each column's 64 rows are one coalesced load), then every wavefront
// multiplies its own upper 16x16 block pairs with v_mfma_f64_16x16x4f64 over
// the panel's 16 groups of 4 rows (A = 16 columns x 4 rows, B = 4 rows x 16
// columns; lane l holds P[4g + l/16][16b + l%16]).  Each workgroup writes its
// upper blocks to gpart[b][64][64].
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int GPR = 64;     // rows per LDS panel

template <class T, bool ROWMAJOR>
__global__ __launch_bounds__(BLOCK) void k_gram(const State* st, const T* __restrict__ X, int64_t ldx, int64_t n,
                                                int which, double* __restrict__ gpart) {
    __shared__ double P[GPR][64 + 1];
    __shared__ double s_scale[64];
    if (st->status != 0) return;
    const int c = which == 0 ? min(st->j, st->m) : st->K;
    const double* scale = which == 0 ? st->scale : st->ysc;
    const int nb = (c + 15) >> 4;
    const int npair = nb * (nb + 1) / 2;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cl = lane & 15, rl = lane >> 4;
    // Block pairs (bi <= bj) of this wavefront: pair t for t = wv, wv + 4, ...
    int pbi[3], pbj[3];
    int np = 0;
    for (int bi = 0, t = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj, ++t)
            if (t % (BLOCK / 64) == wv && np < 3) {
                pbi[np] = bi;
                pbj[np] = bj;
                ++np;
            }
    d4 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    // Columns c .. 16 nb - 1 enter the MFMA tiles as zeros; only the c live
    // columns are loaded per panel.
    for (int idx = threadIdx.x; idx < GPR * (nb * 16 - c); idx += BLOCK) P[idx % GPR][c + idx / GPR] = 0.0;
    if ((int)threadIdx.x < 64) s_scale[threadIdx.x] = (int)threadIdx.x < c ? scale[threadIdx.x] : 0.0;
    // Panel element idx (< GPR c) of thread t is idx = t + q BLOCK.  For the
    // column-major basis, all of a thread's loads of a panel go out together
    // into registers, and the next panel's loads are issued before the
    // current one's products, so a panel costs one memory latency, hidden
    // behind the matrix-core work.
    constexpr int PER = GPR * 64 / BLOCK;
    static_assert(PER * BLOCK == GPR * 64, "a panel of 64 columns splits evenly over the threads");
    auto locate = [&](int idx, int& row, int& col) {
        if (ROWMAJOR) {
            row = idx / c;
            col = idx - row * c;
        } else {
            col = idx / GPR;
            row = idx % GPR;
        }
    };
    T raw[PER];
    auto load_panel = [&](int64_t pn) {
        const int64_t r0 = pn * GPR;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = (int)threadIdx.x + q * BLOCK;
            T v = T(0);
            if (idx < GPR * c) {
                int row = 0, col = 0;
                locate(idx, row, col);
                const int64_t r = r0 + row;
                if (r < n) v = ROWMAJOR ? X[r * ldx + col] : X[(int64_t)col * ldx + r];
            }
            raw[q] = v;
        }
    };
    auto store_panel = [&](int64_t pn) {
        const int64_t r0 = pn * GPR;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = (int)threadIdx.x + q * BLOCK;
            if (idx < GPR * c) {
                int row = 0, col = 0;
                locate(idx, row, col);
                double v = 0.0;
                if (r0 + row < n) v = to_d(raw[q]) * s_scale[col];
                P[row][col] = v;
            }
        }
    };
    const int64_t npanel = (n + GPR - 1) / GPR;
    // The row-major Ritz block (K <= 16 columns, a few loads per thread)
    // measured faster without the prefetch (R-MAT 26: 2.4 against 3.2 ms), so
    // it loads each panel in place; both forms stage the same values.
    if (!ROWMAJOR && (int64_t)blockIdx.x < npanel) load_panel(blockIdx.x);
    for (int64_t pn = blockIdx.x; pn < npanel; pn += gridDim.x) {
        __syncthreads();                 // P is no longer read by the previous panel's products
        if (ROWMAJOR) {
            const int64_t r0 = pn * GPR;
            for (int idx = threadIdx.x; idx < GPR * c; idx += BLOCK) {
                int row = 0, col = 0;
                locate(idx, row, col);
                const int64_t r = r0 + row;
                double v = 0.0;
                if (r < n) v = to_d(X[r * ldx + col]) * s_scale[col];
                P[row][col] = v;
            }
        } else {
            store_panel(pn);
        }
        __syncthreads();
        if (!ROWMAJOR && pn + gridDim.x < npanel) load_panel(pn + gridDim.x);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t < np) {
                const int bi = pbi[t], bj = pbj[t];
#pragma unroll 4
                for (int g = 0; g < GPR / 4; ++g) {
                    const double a = P[g * 4 + rl][bi * 16 + cl];
                    const double b = P[g * 4 + rl][bj * 16 + cl];
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    }
    double* gp = gpart + (int64_t)blockIdx.x * 64 * 64;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (t < np)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // Accumulator element e of lane l holds D[4e + l/16][l % 16].
                const int i = pbi[t] * 16 + e * 4 + rl, jj = pbj[t] * 16 + cl;
                gp[i * 64 + jj] = acc[t][e];
            }
    (void)npair;
}

// G[i][j] = sum over workgroups of the upper blocks, symmetrised: one
// wavefront per entry, lane-strided over the workgroups, then the butterfly
// (a fixed order).
__global__ __launch_bounds__(BLOCK) void k_gram_reduce(const State* st, const double* gpart, int nparts, int which,
                                                       double* G) {
    const int c = which == 0 ? min(st->j, st->m) : st->K;
    const int lane = threadIdx.x & 63;
    const int entry = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    if (entry >= 64 * 64) return;
    const int i = entry / 64, jj = entry % 64;
    if (i >= c || jj >= c || i > jj) return;
    double s = 0.0;
    for (int b = lane; b < nparts; b += 64) s += gpart[(int64_t)b * 4096 + i * 64 + jj];
    s = wave_sum(s);
    if (lane == 0) {
        G[i * 64 + jj] = s;
        G[jj * 64 + i] = s;
    }
}

// max |G - I| and, for the Ritz vectors, the mean angle between pairs.
__global__ __launch_bounds__(BLOCK) void k_gram_metrics(State* st, const double* G, int which) {
    __shared__ double shd[BLOCK / 64];
    __shared__ double shm[BLOCK];
    if (st->status != 0) return;
    const int c = which == 0 ? min(st->j, st->m) : st->K;
    double worst = 0.0, ang = 0.0;
    for (int idx = threadIdx.x; idx < c * c; idx += BLOCK) {
        const int i = idx / c, jj = idx % c;
        const double g = G[i * 64 + jj];
        worst = fmax(worst, fabs(g - (i == jj ? 1.0 : 0.0)));
        if (i < jj) ang += acos(fmin(1.0, fabs(g))) * (180.0 / 3.14159265358979323846);
    }
    shm[threadIdx.x] = worst;
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + o]);
        __syncthreads();
    }
    ang = block_sum(ang, shd);
    if (threadIdx.x == 0) {
        if (which == 0) {
            st->ortho_loss = shm[0];
        } else {
            st->ritz_ortho_loss = shm[0];
            st->mean_angle_deg = c > 1 ? ang / (0.5 * c * (c - 1)) : 90.0;
        }
    }
}

// ---------------------------------------------------------------- launchers
static int pow2_at_least(int k) {
    int v = 1;
    while (v < k) v <<= 1;
    return v;
}

static int gram_grid(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(GRAM_PARTS, (n + GPR - 1) / GPR));
}

template <int P>
static hipError_t finish_p(const Plan& p, const Bufs& b, const Csr& a, double* out_vals, double* out_vecs,
                           int report, hipStream_t s) {
    using VT = typename Tr<P>::V;
    const VT* V = (const VT*)b.V;
    hipLaunchKernelGGL(k_jacobi_select, dim3(1), dim3(JBLOCK), 0, s, b.st, out_vals, p.strict_m);
    switch (p.KB) {
#define LZ_RITZ_CASE(KBV)                                                                                    \
    case KBV:                                                                                                \
        hipLaunchKernelGGL((k_ritz<P, KBV>), dim3(p.g_dense), dim3(BLOCK), 0, s, b.st, V, p.n, p.ld, b.Y);  \
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
    const int kb2 = pow2_at_least(p.K);
    const int gc = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (p.n * kb2 + 4 * BLOCK - 1) / (4 * BLOCK)));
    hipLaunchKernelGGL(k_colstats, dim3(gc), dim3(BLOCK), 0, s, b.st, b.Y, p.n, kb2, b.part);
    if (report && p.ooc) {
        // Host-resident matrix: the residual product streams the slabs too.
        const hipError_t e = ooc_pass(*p.ooc, b.st, s,
                                      [&](const int32_t* col, const void* val, int64_t tb, int64_t te, int, int) {
                                          hipLaunchKernelGGL((k_spmm<P>), dim3(p.g_slab), dim3(BLOCK), 0, s, b.st,
                                                             b.Y, b.Z, p.n, p.nnz, p.n_tiles, b.ob, b.tk, b.head,
                                                             b.tail, kb2, a.rowptr, col, val, nullptr, nullptr,
                                                             nullptr, tb, te);
                                      });
        if (e != hipSuccess) return e;
    } else if (report) {
        hipLaunchKernelGGL((k_spmm<P>), dim3(p.g_tile), dim3(BLOCK), 0, s, b.st, b.Y, b.Z, p.n, p.nnz, p.n_tiles,
                           b.ob, b.tk, b.head, b.tail, kb2, a.rowptr, a.col, a.val, b.rp2, b.col2, b.val2,
                           (int64_t)0, p.n_tiles);
    }
    const int go = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (p.n + 63) / 64));
    hipLaunchKernelGGL(k_out, dim3(go), dim3(BLOCK), 0, s, b.st, b.Y, p.n, kb2, out_vecs);
    if (!report) return hipGetLastError();
    hipLaunchKernelGGL(k_resid, dim3(gc), dim3(BLOCK), 0, s, b.st, b.Y, b.Z, p.n, kb2, b.part2);
    const int gg = gram_grid(p.n);
    double* G = b.gram + (int64_t)GRAM_PARTS * 4096;
    hipLaunchKernelGGL((k_gram<VT, false>), dim3(gg), dim3(BLOCK), 0, s, b.st, V, p.ld, p.n, 0, b.gram);
    hipLaunchKernelGGL(k_gram_reduce, dim3(64 * 64 / (BLOCK / 64)), dim3(BLOCK), 0, s, b.st, b.gram, gg, 0, G);
    hipLaunchKernelGGL(k_gram_metrics, dim3(1), dim3(BLOCK), 0, s, b.st, G, 0);
    hipLaunchKernelGGL((k_gram<double, true>), dim3(gg), dim3(BLOCK), 0, s, b.st, b.Y, (int64_t)p.K, p.n, 1, b.gram);
    hipLaunchKernelGGL(k_gram_reduce, dim3(64 * 64 / (BLOCK / 64)), dim3(BLOCK), 0, s, b.st, b.gram, gg, 1, G);
    hipLaunchKernelGGL(k_gram_metrics, dim3(1), dim3(BLOCK), 0, s, b.st, G, 1);
    return hipGetLastError();
}

hipError_t launch_finish(const Plan& p, const Bufs& b, const Csr& a, double* out_vals, double* out_vecs, int report,
                         hipStream_t s) {
    switch (p.prec) {
        case 0: return finish_p<0>(p, b, a, out_vals, out_vecs, report, s);
        case 1: return finish_p<1>(p, b, a, out_vals, out_vecs, report, s);
        case 2: return finish_p<2>(p, b, a, out_vals, out_vecs, report, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gram_only(int prec, const void* X, int64_t ldx, int64_t n, State* st, double* gram,
                            hipStream_t s) {
    const int gg = gram_grid(n);
    double* G = gram + (int64_t)GRAM_PARTS * 4096;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL((k_gram<double, false>), dim3(gg), dim3(BLOCK), 0, s, st, (const double*)X, ldx, n, 0,
                               gram);
            break;
        case 1:
            hipLaunchKernelGGL((k_gram<float, false>), dim3(gg), dim3(BLOCK), 0, s, st, (const float*)X, ldx, n, 0,
                               gram);
            break;
        case 2:
            hipLaunchKernelGGL((k_gram<uint16_t, false>), dim3(gg), dim3(BLOCK), 0, s, st, (const uint16_t*)X, ldx,
                               n, 0, gram);
            break;
        default:
            return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_gram_reduce, dim3(64 * 64 / (BLOCK / 64)), dim3(BLOCK), 0, s, st, gram, gg, 0, G);
    hipLaunchKernelGGL(k_gram_metrics, dim3(1), dim3(BLOCK), 0, s, st, G, 0);
    return hipGetLastError();
}

hipError_t launch_jacobi_only(const double* alpha, const double* offdiag, int m, State* st, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_only, dim3(1), dim3(JBLOCK), 0, s, alpha, offdiag, m, st);
    return hipGetLastError();
}

}  // namespace lz
