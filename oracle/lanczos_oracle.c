/*
 * FP64 CPU oracle for the Top-K sparse eigensolver (Lanczos + Jacobi),
 * "A Mixed Precision, Multi-GPU Design for Large-scale Top-K Sparse
 * Eigenproblems" (Sgherzi, Parravicini, Santambrogio, 2022).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, sequential
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links or calls it, and it shares no code, header or
 * table with the HIP sources.
 *
 * Every floating-point operation is IEEE binary64, every sum runs in index
 * order, and nothing is blocked, fused or reordered beyond what the paper's
 * Algorithm 1 and the Jacobi method state.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - The loop runs m >= K steps and keeps the K Ritz pairs largest in
 *     modulus (Sec. I names "largest in modulo"; Algorithm 1 runs K steps,
 *     which is the special case m = K).
 *   - beta_1 = 0, beta_i = ||v_nxt|| at the top of step i; the off-diagonal
 *     entries of T are beta_2..beta_m (Algorithm 1 returns a list that is one
 *     short and mis-indexed as printed).
 *   - The orthogonalisation loop of Algorithm 1 (a ping-pong between two
 *     buffers) is read as modified Gram-Schmidt of v_nxt against
 *     v_1..v_i.  `passes` sets how often it is applied: 1 is the paper's
 *     single pass, 2 (default) is "twice is enough", 0 disables it.
 *   - alpha_i = v_i . (M v_i) is taken before the three-term update and the
 *     orthogonalisation (Algorithm 1, the alpha line precedes both).
 *   - Breakdown (beta_i <= tau, an invariant subspace was found): T gets a
 *     zero off-diagonal entry and a fresh random vector, orthogonalised
 *     twice against the basis, continues the iteration.
 *     tau = 100 * unit_roundoff * max_{j<i} (|alpha_j| + beta_j).
 *   - The start vector is u_r = U01(SplitMix64(seed, r)), v_1 = u/||u||;
 *     restart number k draws from seed + k * 2^32.
 *   - Jacobi is the cyclic-by-row method with Rutishauser's rotation
 *     (Sec. III cites Rutishauser's Jacobi method for the small problem).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Progress lines on stderr, one per Lanczos step (long runs on large
 * matrices); no effect on any result. */
static int orc_progress = 0;
void orc_set_progress(int on) { orc_progress = on; }

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  The state after k steps is seed + k*gamma, so
 * output number r (0-based) of the stream started at `seed` is the mix of
 * seed + (r+1)*gamma.                                                       */
uint64_t orc_splitmix64(uint64_t seed, uint64_t r)
{
    uint64_t z = seed + (r + 1u) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Uniform double in [0, 1): the top 53 bits of the output scaled by 2^-53. */
double orc_u01(uint64_t seed, uint64_t r)
{
    return (double)(orc_splitmix64(seed, r) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Dense vector helpers (sequential index order).                           */
static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t r = 0; r < n; ++r) s += a[r] * b[r];
    return s;
}

static double nrm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

/* y = M x for a CSR matrix (Algorithm 1, the SpMV line). */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col,
              const double *val, const double *x, double *y)
{
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) s += val[k] * x[col[k]];
        y[r] = s;
    }
}

/* Modified Gram-Schmidt of w against the columns v_1..v_cnt of V (n rows,
 * column j at V + j*n), repeated `passes` times (Algorithm 1, the
 * orthogonalisation loop). */
static void mgs(int64_t n, const double *V, int cnt, double *w, int passes)
{
    for (int p = 0; p < passes; ++p)
        for (int j = 0; j < cnt; ++j) {
            const double *vj = V + (int64_t)j * n;
            double o = dot(n, vj, w);
            for (int64_t r = 0; r < n; ++r) w[r] -= o * vj[r];
        }
}

/*
 * The start vector v_1 = u/||u||, u_r = U01(SplitMix64(seed, r)) (Algorithm 1
 * takes an L2-normalised random vector), as orc_lanczos computes it.
 */
void orc_start_vector(int64_t n, uint64_t seed, double *v)
{
    for (int64_t r = 0; r < n; ++r) v[r] = orc_u01(seed, (uint64_t)r);
    double s = nrm2(n, v);
    for (int64_t r = 0; r < n; ++r) v[r] /= s;
}

/*
 * Lanczos with full reorthogonalisation (Algorithm 1), m steps.
 *
 * Outputs (1-based paper indices stored 0-based):
 *   alpha[i-1] = alpha_i, i = 1..m
 *   beta[i-1]  = beta_i,  i = 1..m+1  (beta_1 = 0; beta_{m+1} = ||v_nxt||
 *                after the last step, used by residual estimates)
 *   V[(i-1)*n + r] = v_i[r], i = 1..m+1 (column v_{m+1} is zero when
 *                beta_{m+1} = 0).  V must hold n*(m+1) doubles.
 * Returns the number of restarts after breakdown, or -1 on bad arguments,
 * -2 when a restart vector is itself numerically in the span of the basis.
 */
int orc_lanczos(int64_t n, const int64_t *rowptr, const int32_t *col,
                const double *val, int m, uint64_t seed, int passes,
                double unit_roundoff, double *alpha, double *beta, double *V)
{
    if (n < 1 || m < 1 || m > n || passes < 0 || !alpha || !beta || !V) return -1;
    double *vt = (double *)malloc(sizeof(double) * (size_t)n);   /* v_tmp */
    double *vn = (double *)malloc(sizeof(double) * (size_t)n);   /* v_nxt */
    if (!vt || !vn) { free(vt); free(vn); return -1; }

    int restarts = 0;
    double tnorm = 0.0;      /* running max_j (|alpha_j| + beta_j) */

    /* v_1: L2-normalised random vector (Sec. III, Algorithm 1 inputs). */
    double *v1 = V;
    for (int64_t r = 0; r < n; ++r) v1[r] = orc_u01(seed, (uint64_t)r);
    double s0 = nrm2(n, v1);
    for (int64_t r = 0; r < n; ++r) v1[r] /= s0;
    beta[0] = 0.0;                                              /* beta_1 */

    for (int i = 1; i <= m; ++i) {
        double *vi = V + (int64_t)(i - 1) * n;
        if (i != 1) {
            /* Normalise and compute the new Lanczos vector. */
            double b = nrm2(n, vn);
            double tau = 100.0 * unit_roundoff * tnorm;
            if (!(b > tau)) {
                /* Breakdown: Krylov space invariant; restart with a fresh
                 * random vector orthogonal to v_1..v_{i-1}. */
                ++restarts;
                uint64_t rs = seed + ((uint64_t)restarts << 32);
                for (int64_t r = 0; r < n; ++r) vn[r] = orc_u01(rs, (uint64_t)r);
                mgs(n, V, i - 1, vn, 2);
                double bn = nrm2(n, vn);
                if (!(bn > 0.0)) { free(vt); free(vn); return -2; }
                for (int64_t r = 0; r < n; ++r) vi[r] = vn[r] / bn;
                beta[i - 1] = 0.0;
            } else {
                beta[i - 1] = b;
                for (int64_t r = 0; r < n; ++r) vi[r] = vn[r] / b;
            }
        }
        /* Compute the next projection. */
        orc_spmv(n, rowptr, col, val, vi, vt);                 /* v_t = M v_i */
        double a = dot(n, vi, vt);                              /* alpha_i */
        alpha[i - 1] = a;
        const double *vprev = (i >= 2) ? V + (int64_t)(i - 2) * n : NULL;
        double bi = beta[i - 1];
        for (int64_t r = 0; r < n; ++r)
            vn[r] = vt[r] - a * vi[r] - (vprev ? bi * vprev[r] : 0.0);
        mgs(n, V, i, vn, passes);                               /* orthogonalise */
        double t = fabs(a) + bi;
        if (t > tnorm) tnorm = t;
        if (orc_progress) { fprintf(stderr, "oracle: Lanczos step %d/%d\n", i, m); fflush(stderr); }
    }
    /* beta_{m+1} and v_{m+1} (residual estimate only). */
    double bl = nrm2(n, vn);
    beta[m] = bl;
    double *vl = V + (int64_t)m * n;
    for (int64_t r = 0; r < n; ++r) vl[r] = (bl > 0.0) ? vn[r] / bl : 0.0;
    free(vt);
    free(vn);
    return restarts;
}

/*
 * Cyclic-by-row Jacobi eigensolver for a dense symmetric m x m matrix
 * (Sec. III, the second phase; Rutishauser's formulation).
 *   A: row-major, overwritten; on return its diagonal holds the eigenvalues.
 *   S: row-major m x m; on return column k is the eigenvector of A_kk.
 * A rotation in plane (p,q) is skipped when |a_pq| is negligible against
 * the diagonal (|a_pq| <= eps*sqrt(|a_pp a_qq|)) or against the matrix
 * (|a_pq| <= eps^2 * ||A||_F).  The method stops after a sweep that applied
 * no rotation.  Returns the number of sweeps, or -1 if max_sweeps ran out.
 */
int orc_jacobi(int m, double *A, double *S, int max_sweeps)
{
    const double eps = 1.1102230246251565e-16;                 /* 2^-53 */
    double fro = 0.0;
    for (int k = 0; k < m * m; ++k) fro += A[k] * A[k];
    fro = sqrt(fro);
    for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q) S[p * m + q] = (p == q) ? 1.0 : 0.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < m - 1; ++p) {
            for (int q = p + 1; q < m; ++q) {
                double apq = A[p * m + q];
                double app = A[p * m + p], aqq = A[q * m + q];
                if (fabs(apq) <= eps * sqrt(fabs(app * aqq)) || fabs(apq) <= eps * eps * fro)
                    continue;
                /* t = tan of the rotation angle, the root of
                 * t^2 + 2 zeta t - 1 = 0 of smaller modulus. */
                double zeta = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(zeta) > 1e150)
                    t = 0.5 / zeta;
                else
                    t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                A[p * m + p] = app - t * apq;
                A[q * m + q] = aqq + t * apq;
                A[p * m + q] = 0.0;
                A[q * m + p] = 0.0;
                for (int r = 0; r < m; ++r) {
                    if (r == p || r == q) continue;
                    double arp = A[r * m + p], arq = A[r * m + q];
                    double np = c * arp - s * arq;
                    double nq = s * arp + c * arq;
                    A[r * m + p] = np; A[p * m + r] = np;
                    A[r * m + q] = nq; A[q * m + r] = nq;
                }
                for (int r = 0; r < m; ++r) {
                    double srp = S[r * m + p], srq = S[r * m + q];
                    S[r * m + p] = c * srp - s * srq;
                    S[r * m + q] = s * srp + c * srq;
                }
                rotated = 1;
            }
        }
        if (!rotated) return sweep;
    }
    return -1;
}

/*
 * Top-K selection (Sec. I: the eigenvalues largest in modulus).  Order:
 * |theta| descending, then theta descending, then index ascending.
 * idx receives K indices into theta.
 */
void orc_select_topk(int m, const double *theta, int K, int *idx)
{
    int *ord = (int *)malloc(sizeof(int) * (size_t)m);
    for (int i = 0; i < m; ++i) ord[i] = i;
    for (int i = 1; i < m; ++i) {            /* insertion sort, stable */
        int cur = ord[i];
        int j = i - 1;
        while (j >= 0) {
            double a = theta[ord[j]], b = theta[cur];
            int before = (fabs(b) > fabs(a)) || (fabs(b) == fabs(a) && b > a);
            if (!before) break;
            ord[j + 1] = ord[j];
            --j;
        }
        ord[j + 1] = cur;
    }
    for (int k = 0; k < K; ++k) idx[k] = ord[k];
    free(ord);
}

/*
 * Ritz vectors (Sec. III: the eigenvectors of M are the Lanczos basis times
 * the eigenvectors of T).  Y[:,k] = sum_i V[:,i] * S[i, idx[k]], i < m,
 * then scaled to unit 2-norm and signed so that its entry of largest
 * modulus (lowest index on ties) is positive.  Y is n x K column-major.
 */
void orc_ritz(int64_t n, int m, const double *V, const double *S, int K,
              const int *idx, double *Y)
{
    for (int k = 0; k < K; ++k) {
        double *y = Y + (int64_t)k * n;
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += V[(int64_t)i * n + r] * S[i * m + idx[k]];
            y[r] = s;
        }
        double nr = nrm2(n, y);
        int64_t amax = 0;
        for (int64_t r = 1; r < n; ++r)
            if (fabs(y[r]) > fabs(y[amax])) amax = r;
        double sc = (y[amax] < 0.0 ? -1.0 : 1.0) / nr;
        for (int64_t r = 0; r < n; ++r) y[r] *= sc;
    }
}

/*
 * Accuracy report (Sec. IV-D): for each Ritz pair the absolute residual
 * ||M y - theta y|| (the paper's L2 reconstruction error) and the relative
 * one, divided by |theta| (equal to the absolute one when theta = 0).
 */
void orc_residuals(int64_t n, const int64_t *rowptr, const int32_t *col,
                   const double *val, int K, const double *vals, const double *Y,
                   double *abs_resid, double *rel_resid)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    for (int k = 0; k < K; ++k) {
        const double *y = Y + (int64_t)k * n;
        orc_spmv(n, rowptr, col, val, y, t);
        double s = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double d = t[r] - vals[k] * y[r];
            s += d * d;
        }
        abs_resid[k] = sqrt(s);
        /* Relative to |theta|; an exact zero Ritz value has no scale, so its
         * relative residual is the absolute one. */
        rel_resid[k] = vals[k] != 0.0 ? sqrt(s) / fabs(vals[k]) : sqrt(s);
    }
    free(t);
}

/* max_{i,j} |(X^T X - I)_{ij}| for the first c columns of X (n rows). */
double orc_ortho_loss(int64_t n, int c, const double *X)
{
    double worst = 0.0;
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) {
            double g = dot(n, X + (int64_t)i * n, X + (int64_t)j * n);
            double e = fabs(g - (i == j ? 1.0 : 0.0));
            if (e > worst) worst = e;
        }
    return worst;
}

/* The paper's orthogonality metric (Sec. IV-D): the mean angle, in
 * degrees, between every pair of eigenvectors (90 is ideal). */
double orc_mean_angle_deg(int64_t n, int K, const double *Y)
{
    if (K < 2) return 90.0;
    double s = 0.0;
    int cnt = 0;
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j) {
            double g = fabs(dot(n, Y + (int64_t)i * n, Y + (int64_t)j * n));
            if (g > 1.0) g = 1.0;
            s += acos(g) * (180.0 / 3.14159265358979323846);
            ++cnt;
        }
    return s / cnt;
}

/* ------------------------------------------------------------------------ */
/* Precision emulation (Sec. III-A: vectors stored in a narrower format than
 * the arithmetic).  Not part of the FP64 definition above: it re-runs
 * Algorithm 1 with the stored quantities rounded, to predict how much a
 * reduced storage precision moves the results, so that precision loss can be
 * told apart from implementation errors.                                   */

/* x rounded to the nearest number with `bits` significant bits (ties to the
 * even significand).  bits >= 53 returns x; 24 gives the binary32 value and
 * 8 the bfloat16 value of a double in their normal ranges. */
double orc_round_bits(double x, int bits)
{
    if (bits >= 53 || x == 0.0 || !isfinite(x)) return x;
    int e;
    double f = frexp(x, &e);                  /* x = f * 2^e, 0.5 <= |f| < 1 */
    double sig = ldexp(f, bits);              /* |sig| in [2^(bits-1), 2^bits) */
    double r = floor(sig);
    double d = sig - r;
    if (d > 0.5 || (d == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
    return ldexp(r, e - bits);
}

/* y = M x with every product and every partial sum rounded to acc_bits
 * (the SpMV of a reduced-precision accumulator), rows summed in entry
 * order. */
void orc_spmv_emul(int64_t n, const int64_t *rowptr, const int32_t *col,
                   const double *val, const double *x, double *y, int acc_bits)
{
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
            s = orc_round_bits(s + orc_round_bits(val[k] * x[col[k]], acc_bits), acc_bits);
        y[r] = s;
    }
}

/* v = round(w) / ||round(w)||: a Lanczos vector as stored in the basis
 * precision, scaled to unit length in binary64.  Returns ||round(w)||. */
static double store_unit(int64_t n, const double *w, double *v, int store_bits)
{
    for (int64_t r = 0; r < n; ++r) v[r] = orc_round_bits(w[r], store_bits);
    double b = nrm2(n, v);
    if (b > 0.0)
        for (int64_t r = 0; r < n; ++r) v[r] /= b;
    return b;
}

/*
 * Algorithm 1 as orc_lanczos, with three roundings a mixed-precision run
 * applies: every Lanczos vector is stored rounded to store_bits (then used
 * at unit length), the SpMV products and sums are rounded to acc_bits, and
 * its output is held in a working vector rounded to work_bits.  The dots,
 * the three-term update and the Gram-Schmidt passes stay binary64.  With
 * all three >= 53 every rounding is the identity and the results equal
 * orc_lanczos bit for bit.  Same arguments, outputs and return codes.
 */
int orc_lanczos_emul(int64_t n, const int64_t *rowptr, const int32_t *col,
                     const double *val, int m, uint64_t seed, int passes,
                     double unit_roundoff, int store_bits, int acc_bits, int work_bits,
                     double *alpha, double *beta, double *V)
{
    if (n < 1 || m < 1 || m > n || passes < 0 || !alpha || !beta || !V) return -1;
    double *vt = (double *)malloc(sizeof(double) * (size_t)n);
    double *vn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!vt || !vn) { free(vt); free(vn); return -1; }

    int restarts = 0;
    double tnorm = 0.0;

    for (int64_t r = 0; r < n; ++r) vn[r] = orc_u01(seed, (uint64_t)r);
    store_unit(n, vn, V, store_bits);                          /* v_1 */
    beta[0] = 0.0;

    for (int i = 1; i <= m; ++i) {
        double *vi = V + (int64_t)(i - 1) * n;
        if (i != 1) {
            double *tmp = vt;                  /* stored candidate for v_i */
            for (int64_t r = 0; r < n; ++r) tmp[r] = orc_round_bits(vn[r], store_bits);
            double b = nrm2(n, tmp);
            double tau = 100.0 * unit_roundoff * tnorm;
            if (!(b > tau)) {
                ++restarts;
                uint64_t rs = seed + ((uint64_t)restarts << 32);
                for (int64_t r = 0; r < n; ++r) vn[r] = orc_u01(rs, (uint64_t)r);
                mgs(n, V, i - 1, vn, 2);
                double bn = store_unit(n, vn, vi, store_bits);
                if (!(bn > 0.0)) { free(vt); free(vn); return -2; }
                beta[i - 1] = 0.0;
            } else {
                beta[i - 1] = b;
                for (int64_t r = 0; r < n; ++r) vi[r] = tmp[r] / b;
            }
        }
        orc_spmv_emul(n, rowptr, col, val, vi, vt, acc_bits);    /* v_t = M v_i */
        for (int64_t r = 0; r < n; ++r) vt[r] = orc_round_bits(vt[r], work_bits);
        double a = dot(n, vi, vt);
        alpha[i - 1] = a;
        const double *vprev = (i >= 2) ? V + (int64_t)(i - 2) * n : NULL;
        double bi = beta[i - 1];
        for (int64_t r = 0; r < n; ++r)
            vn[r] = vt[r] - a * vi[r] - (vprev ? bi * vprev[r] : 0.0);
        mgs(n, V, i, vn, passes);
        double t = fabs(a) + bi;
        if (t > tnorm) tnorm = t;
        if (orc_progress) { fprintf(stderr, "oracle (emulated): Lanczos step %d/%d\n", i, m); fflush(stderr); }
    }
    double *vl = V + (int64_t)m * n;
    double bl = store_unit(n, vn, vl, store_bits);
    beta[m] = bl;
    if (!(bl > 0.0))
        for (int64_t r = 0; r < n; ++r) vl[r] = 0.0;
    free(vt);
    free(vn);
    return restarts;
}
