// Seeded synthetic sparse symmetric matrices (CSR) standing in for the
// paper's graph workloads (Table I: SuiteSparse web/social/road graphs and
// the GAP kron/urand graphs).  Two families:
//
//   * Erdos-Renyi G(n, p) over the strict upper triangle, mirrored, with
//     uniform(-1,1) off-diagonal values and a uniform(0,1) diagonal.
//     Edges are drawn row by row with geometric skipping (Batagelj and
//     Brandes, "Efficient generation of large random networks", 2005).
//   * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) with quadrant
//     probabilities a, b, c, d: each edge picks one quadrant per bit level.
//     Self loops are dropped, edges are made undirected and deduplicated,
//     weights are uniform(0,1) per unordered pair, vertex ids are optionally
//     relabelled by a seeded random permutation.
//
// Every random draw is a SplitMix64 output (Steele, Lea, Flood 2014) taken
// at a counter that names what it is for, so the output does not depend on
// the number of threads.  This module holds no eigensolver arithmetic; it is
// shared by the tests, the benchmark and the serving driver to make inputs.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <parallel/algorithm>
#include <vector>

#include <omp.h>

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
// Output number r (0-based) of the SplitMix64 stream started at `seed`.
inline uint64_t sm64(uint64_t seed, uint64_t r) { return mix64(seed + (r + 1) * kGamma); }
inline double u01(uint64_t seed, uint64_t r) {
    return double(sm64(seed, r) >> 11) * (1.0 / 9007199254740992.0);
}
// Distinct sub-stream seeds for the different uses of randomness.
inline uint64_t substream(uint64_t seed, uint64_t tag) { return mix64(seed ^ mix64(tag * kGamma + 0x1234567ULL)); }

enum : uint64_t { TAG_ER_ROW = 1, TAG_ER_OFF = 2, TAG_ER_DIAG = 3, TAG_RMAT_EDGE = 4,
                  TAG_RMAT_W = 5, TAG_PERM = 6 };

// Builds a symmetric CSR from an undirected edge list (u != v, each pair
// once) plus an optional dense diagonal.  Rows come out with sorted columns.
void build_sym_csr(int64_t n, const std::vector<uint32_t>& eu, const std::vector<uint32_t>& ev,
                   const std::vector<double>& ew, const double* diag,
                   int64_t* rowptr, int32_t* col, double* val) {
    const int64_t E = (int64_t)eu.size();
    std::vector<std::atomic<int64_t>> cnt(n);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) cnt[r].store(diag ? 1 : 0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        cnt[eu[e]].fetch_add(1, std::memory_order_relaxed);
        cnt[ev[e]].fetch_add(1, std::memory_order_relaxed);
    }
    rowptr[0] = 0;
    for (int64_t r = 0; r < n; ++r) rowptr[r + 1] = rowptr[r] + cnt[r].load();
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        int64_t p = rowptr[r];
        if (diag) { col[p] = (int32_t)r; val[p] = diag[r]; ++p; }
        cnt[r].store(p, std::memory_order_relaxed);
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        int64_t pu = cnt[eu[e]].fetch_add(1, std::memory_order_relaxed);
        col[pu] = (int32_t)ev[e]; val[pu] = ew[e];
        int64_t pv = cnt[ev[e]].fetch_add(1, std::memory_order_relaxed);
        col[pv] = (int32_t)eu[e]; val[pv] = ew[e];
    }
    // Sort every row by column (columns are unique within a row).
#pragma omp parallel
    {
        std::vector<std::pair<int32_t, double>> buf;
#pragma omp for schedule(dynamic, 1024)
        for (int64_t r = 0; r < n; ++r) {
            int64_t b = rowptr[r], e = rowptr[r + 1];
            buf.resize(e - b);
            for (int64_t k = b; k < e; ++k) buf[k - b] = {col[k], val[k]};
            std::sort(buf.begin(), buf.end(),
                      [](const auto& x, const auto& y) { return x.first < y.first; });
            for (int64_t k = b; k < e; ++k) { col[k] = buf[k - b].first; val[k] = buf[k - b].second; }
        }
    }
}

struct Graph {
    int64_t n = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

}  // namespace

extern "C" {

// Handle-based API: generate into an internal buffer, query sizes, copy out.
void* syn_er(int64_t n, double offdiag_per_row, uint64_t seed) {
    if (n < 1) return nullptr;
    auto* g = new Graph;
    g->n = n;
    const double p = (n > 1) ? std::min(1.0, offdiag_per_row / double(n - 1)) : 0.0;
    const uint64_t srow = substream(seed, TAG_ER_ROW), soff = substream(seed, TAG_ER_OFF),
                   sdiag = substream(seed, TAG_ER_DIAG);
    // Pass 1: count the upper-triangle edges of every row; pass 2: emit them.
    std::vector<int64_t> cnt(n + 1, 0);
    auto walk = [&](int64_t i, auto&& emit) {
        if (p <= 0.0) return;
        const uint64_t rs = sm64(srow, (uint64_t)i);
        const double lq = std::log1p(-p);
        int64_t j = i;
        for (uint64_t k = 0;; ++k) {
            double u = u01(rs, k);
            int64_t skip = (p >= 1.0) ? 0 : (int64_t)std::floor(std::log1p(-u) / lq);
            j += 1 + skip;
            if (j >= n || j < 0) break;
            emit(j);
        }
    };
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        walk(i, [&](int64_t) { ++c; });
        cnt[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<uint32_t> eu(cnt[n]), ev(cnt[n]);
    std::vector<double> ew(cnt[n]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t pos = cnt[i];
        walk(i, [&](int64_t j) {
            eu[pos] = (uint32_t)i; ev[pos] = (uint32_t)j;
            ew[pos] = 2.0 * u01(soff, (uint64_t)i * (uint64_t)n + (uint64_t)j) - 1.0;
            ++pos;
        });
    }
    std::vector<double> diag(n);
    for (int64_t i = 0; i < n; ++i) diag[i] = u01(sdiag, (uint64_t)i);
    g->rowptr.resize(n + 1);
    const int64_t nnz = n + 2 * cnt[n];
    g->col.resize(nnz);
    g->val.resize(nnz);
    build_sym_csr(n, eu, ev, ew, diag.data(), g->rowptr.data(), g->col.data(), g->val.data());
    return g;
}

// R-MAT over 2^scale vertices truncated to n (edges with an endpoint >= n
// are redrawn), n_edges directed draws, quadrant probabilities a, b, c and
// d = 1 - a - b - c.
void* syn_rmat(int64_t n, int scale, int64_t n_edges, double a, double b, double c,
               uint64_t seed, int permute) {
    if (n < 2 || scale < 1 || scale > 31 || (int64_t(1) << scale) < n || n_edges < 0) return nullptr;
    auto* g = new Graph;
    g->n = n;
    const uint64_t se = substream(seed, TAG_RMAT_EDGE), sw = substream(seed, TAG_RMAT_W);
    const double ab = a + b, abc = a + b + c;
    std::vector<uint64_t> keys(n_edges);
    // Draw edge e at attempt t from counter (t * n_edges + e) * 64 + level.
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_edges; ++e) {
        uint64_t key = ~0ULL;
        for (uint64_t t = 0; t < 64; ++t) {
            uint64_t u = 0, v = 0;
            const uint64_t base = (t * (uint64_t)n_edges + (uint64_t)e) * 64;
            for (int l = 0; l < scale; ++l) {
                double r = u01(se, base + (uint64_t)l);
                uint64_t bu, bv;
                if (r < a) { bu = 0; bv = 0; }
                else if (r < ab) { bu = 0; bv = 1; }
                else if (r < abc) { bu = 1; bv = 0; }
                else { bu = 1; bv = 1; }
                u |= bu << (scale - 1 - l);
                v |= bv << (scale - 1 - l);
            }
            if ((int64_t)u < n && (int64_t)v < n) {
                if (u != v) key = (std::min(u, v) << 32) | std::max(u, v);
                break;
            }
        }
        keys[e] = key;
    }
    __gnu_parallel::sort(keys.begin(), keys.end());
    auto last = std::unique(keys.begin(), keys.end());
    if (last != keys.begin() && *(last - 1) == ~0ULL) --last;   // dropped self loops
    const int64_t E = last - keys.begin();
    std::vector<uint32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0u);
    if (permute) {
        const uint64_t sp = substream(seed, TAG_PERM);
        for (int64_t i = n - 1; i > 0; --i) {   // Fisher-Yates
            int64_t j = (int64_t)(u01(sp, (uint64_t)i) * double(i + 1));
            if (j > i) j = i;
            std::swap(perm[i], perm[j]);
        }
    }
    std::vector<uint32_t> eu(E), ev(E);
    std::vector<double> ew(E);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        uint64_t k = keys[e];
        eu[e] = perm[k >> 32];
        ev[e] = perm[k & 0xffffffffULL];
        ew[e] = u01(sw, k);
    }
    std::vector<uint64_t>().swap(keys);
    g->rowptr.resize(n + 1);
    g->col.resize(2 * E);
    g->val.resize(2 * E);
    build_sym_csr(n, eu, ev, ew, nullptr, g->rowptr.data(), g->col.data(), g->val.data());
    return g;
}

int64_t syn_n(void* h) { return h ? ((Graph*)h)->n : -1; }
int64_t syn_nnz(void* h) { return h ? (int64_t)((Graph*)h)->col.size() : -1; }

void syn_copy(void* h, int64_t* rowptr, int32_t* col, double* val) {
    auto* g = (Graph*)h;
    std::memcpy(rowptr, g->rowptr.data(), sizeof(int64_t) * g->rowptr.size());
    std::memcpy(col, g->col.data(), sizeof(int32_t) * g->col.size());
    std::memcpy(val, g->val.data(), sizeof(double) * g->val.size());
}

void syn_free(void* h) { delete (Graph*)h; }

// Symmetric degree normalisation D^{-1/2} A D^{-1/2}, d_i = sum_j a_ij.
// Rows with zero degree stay zero.
void syn_normalize_sym(int64_t n, const int64_t* rowptr, const int32_t* col, double* val) {
    std::vector<double> s(n);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        double d = 0.0;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) d += val[k];
        s[r] = d > 0.0 ? 1.0 / std::sqrt(d) : 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r)
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k) val[k] *= s[r] * s[col[k]];
}

}  // extern "C"
