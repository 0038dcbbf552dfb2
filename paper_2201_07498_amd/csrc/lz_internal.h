// Internal declarations of the gfx950 Lanczos/Jacobi Top-K solver: the
// device-resident solve state, the workspace plan, precision traits and the
// kernel launchers.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lz {

constexpr int MMAX = 64;       // largest m (Lanczos steps); Jacobi tile in LDS
constexpr int NCMAX = 72;      // column bound of the orthogonalisation kernels (m+1 rounded to 8)
constexpr int BLOCK = 256;     // threads per workgroup (4 wave64)
constexpr int TILE = 1024;     // non-zeros per SpMV tile (one wavefront, 16 per lane)
constexpr int LDPAD = 2048;    // basis leading dimension is a multiple of this
constexpr int OGRID = 256;     // orthogonalisation grid cap (workgroups of OBLOCK threads)
constexpr int OBLOCK = 1024;   // orthogonalisation workgroup (16 wave64)
constexpr int DGRID = 1024;    // grid cap of the other dense kernels (workgroups of BLOCK threads)
constexpr int SGRID = 2048;    // SpMV grid cap (workgroups)
constexpr int GRAM_PARTS = 1024; // Gram kernel grid cap (per-workgroup 64x64 partials)
// Column-sorted storage of the relabelled matrix.  State.packed = PACK_TILE
// (n < 2^22): each tile's entries are stored in column order and each column
// word holds (col << PACK_SLOTBITS) | (the entry's position in the tile's row
// order).  PACK_GROUP (n <= 2^20): the same over groups of GROUP_TILES
// consecutive tiles, with GROUP_SLOTBITS-bit positions in the group.
// PACK_SWEEP (large matrices, opt-in below a size threshold): the rows are
// cut into sweep blocks and each block's entries are stored in column order
// with their row inside the block in a separate array (see below).
enum Packing { PACK_NONE = 0, PACK_TILE = 1, PACK_GROUP = 2, PACK_SWEEP = 3 };
constexpr int PACK_SLOTBITS = 10;   // TILE = 2^10 positions
constexpr int PACK_COLBITS = 22;
constexpr uint32_t PACK_SLOTMASK = (1u << PACK_SLOTBITS) - 1u;
constexpr int GROUP_TILES = 4;
constexpr int GROUP_SLOTBITS = 12;  // GROUP_TILES * TILE = 2^12 positions
constexpr int GROUP_COLBITS = 20;
constexpr uint32_t GROUP_SLOTMASK = (1u << GROUP_SLOTBITS) - 1u;
// Sweep blocks: the relabelled matrix walked as one sequence of items, the
// entries of row 0, SW_W items for the end of row 0, the entries of row 1,
// and so on (entry e of row r is item e + SW_W * r); with R rows per block
// (sweep_rows: 4096 in FP64, 2048 in FP32 and BF16) block b is items
// [b * SW_W * R, (b+1) * SW_W * R) and owns the rows whose end starts in it,
// so a block holds at most SW_W * R entries and R owned rows.  Its
// entries are stored sorted by column (by the 128-byte line of x they
// gather, ties in row order), each with its row relative to the block's
// first owned row; the row continuing past the block, if any, comes right
// after the owned ones (so at most R + 1 rows).
constexpr int SW_W = 64;
constexpr int SW_ROWS_MAX = 4096;
constexpr int sweep_rows(int prec) { return prec == 0 ? 4096 : 2048; }
// Sort payload of an entry: (row within its block << SW_POSBITS) | position
// within its block (at most 64 * 4096 = 2^18 entries per block).
constexpr int SW_POSBITS = 18;
static_assert((int64_t)SW_W * 4096 <= (int64_t(1) << SW_POSBITS) && (4096 << SW_POSBITS) > 0, "sweep payload");
// Automatic choice: relabelled matrices whose x takes at least 64 MiB.
// Measured on MI355X, whole solve (K = 8, m = 32) of R-MAT with edge factor
// 16, tiles -> sweep blocks: scale 24 FP32 149 -> 135 ms, FP64 196 -> 180,
// BF16 (x 32 MiB) 118 -> 120; scale 25 FP32 337 -> 280, BF16 249 -> 242,
// FP64 444 -> 366; scale 26 FP32 769 -> 634, BF16 578 -> 520.  At scale 23
// in FP32 (x 32 MiB) the step SpMV was slower in sweep blocks.
constexpr int64_t SWEEP_AUTO_MIN_N = int64_t(1) << 22;
constexpr uint64_t SWEEP_AUTO_MIN_X_BYTES = uint64_t(1) << 26;

enum Mode { MODE_NORMAL = 0, MODE_RESTART = 1 };

// Tickets of the "last workgroup reduces" pattern, one per kernel kind.
enum Ticket { TK_INIT = 0, TK_SPMV, TK_DOT, TK_UPD, TK_STORE, TK_RITZ, TK_RESID, TK_GRAM, TK_COUNT };

// Solve state kept in device memory; every kernel reads the step index and
// coefficients from here, so the host never has to read them back between
// kernels.  Basis column k is stored unnormalised; its unit vector is
// scale[k] * V[:,k].
struct State {
    int32_t j;            // current Lanczos index (0-based): columns 0..j hold v_1..v_{j+1}
    int32_t mode;         // MODE_NORMAL or MODE_RESTART (next SpMV step draws a restart vector)
    int32_t restarts;
    int32_t status;       // lz_status
    int32_t m, K, reorth, second;   // `second`: run the second update of this step
    int32_t n_items, n_long, sweeps;
    int32_t arith;        // LZ_ARITH_FP32: dots, norms, reorthogonalisation and SpMV epilogue in FP32
    int32_t remeasure;    // two-pass modes: this step's second coefficients are re-measured (see k_orth_dot)
    uint32_t ticket[TK_COUNT];
    uint64_t seed;
    double u_s;           // unit roundoff of the stored basis (selective reorthogonalisation)
    double u_w;           // unit roundoff of the working vector and SpMV accumulation (breakdown)
    double tnorm;         // max_j (|alpha_j| + beta_j), scales the breakdown threshold
    double wnorm2;        // ||w'||^2 after the first update (selective second pass)
    // Matrix of the solve: the caller's CSR or its hub-first relabelling.
    const int64_t* crp;
    const int32_t* ccol;
    const void* cval;
    const int32_t* perm;       // relabelled row -> original row (null: identity)
    const int32_t* iperm;      // original row -> relabelled row
    int32_t reorder, reordered;
    int32_t packed, pad2;      // Packing of the relabelled copy
    unsigned long long maxdeg; // longest row of the input
    double alpha[MMAX + 8];
    double beta[MMAX + 8];     // beta[k] couples columns k-1 and k; beta[0] = 0
    double scale[MMAX + 8];
    double c[NCMAX];           // first-pass projection coefficients (already scaled)
    double c2[NCMAX];          // second-pass coefficients
    double theta[MMAX];        // Ritz values (Jacobi order)
    int32_t sel[MMAX];         // Top-K indices into theta
    double ysc[MMAX];          // Ritz column scale: sign / norm
    double abs_resid[MMAX], resid[MMAX];
    double ortho_loss, ritz_ortho_loss, mean_angle_deg, pad1;
    double S[MMAX * MMAX];     // Jacobi eigenvectors, row-major m x m (stride MMAX)
};

// Host copies of the state: the header (step, mode, restarts, status) for
// the restart check, everything but the Jacobi eigenvectors for the report.
constexpr size_t STATE_HEAD_BYTES = 64;
constexpr size_t STATE_REPORT_BYTES = offsetof(State, S);
static_assert(offsetof(State, status) + sizeof(int32_t) <= STATE_HEAD_BYTES, "state header");

struct Ooc;   // host-resident matrix streamed in slabs (lz_ooc.h)

// Workspace layout of one solve.  All offsets are in bytes from the base.
struct Plan {
    int64_t n = 0, nnz = 0, ld = 0;
    int32_t K = 0, m = 0, prec = 0, KB = 0;
    int32_t g_orth = 0, g_dense = 0, g_tile = 0;
    int32_t xcache = 0;         // Lanczos-step SpMV keeps the head of x in LDS: XC_OFF, XC_ON (set once the
                                // row order is known) or XC_GATED (both variants launched; each returns
                                // unless the device's row-order decision selects it)
    int32_t strict_m = 0;       // the finish reports LZ_ERR_RESTART_BUDGET if fewer than m steps completed
    int32_t fff = 0;            // all-FP32 arithmetic (FP32 storage only): float instantiations
    int32_t g_slab = 0;         // grid of the per-slab launches of a host-resident matrix
    int32_t sweep = 0;          // reserve and build the sweep-block copy if the matrix is relabelled
    int32_t sw_bit0 = 0, sw_bit1 = 0;   // column bits the sweep blocks are sorted on
    int64_t sw_nb = 0;          // sweep blocks
    int64_t sw_items = 0;       // items per sweep block (SW_W * sweep_rows)
    size_t sw_sort_bytes = 0;   // scratch of the segmented sort
    Ooc* ooc = nullptr;         // non-null: the matrix entries stay in host memory
    int64_t n_tiles = 0;
    size_t off_state = 0, off_V = 0, off_w = 0, off_part = 0, off_part2 = 0, off_scan = 0, off_bsum = 0,
           off_Y = 0, off_Z = 0, off_gram = 0, off_ob = 0, off_tk = 0, off_head = 0, off_tail = 0, off_rp2 = 0,
           off_col2 = 0, off_val2 = 0, off_perm = 0, off_iperm = 0, off_gm = 0, off_swob = 0, off_swe = 0,
           off_swcol = 0, off_swrl = 0, off_swval = 0, off_swsrc = 0, off_swvin = 0, off_swtmp = 0, off_swq = 0;
    size_t bytes = 0;
};

enum XcacheChoice { XC_OFF = 0, XC_ON = 1, XC_GATED = 2 };

inline size_t storage_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
inline size_t work_bytes(int prec) { return prec == 0 ? 8 : 4; }
inline double unit_roundoff(int prec) {
    return prec == 0 ? 1.1102230246251565e-16 : (prec == 1 ? 5.9604644775390625e-08 : 3.90625e-03);
}
// The working vector and the SpMV accumulator are FP64 in FP64 mode and FP32
// in both mixed modes.
inline double work_roundoff(int prec) { return prec == 0 ? 1.1102230246251565e-16 : 5.9604644775390625e-08; }

// `relabel`: reserve the hub-first relabelled copy of the matrix (without it
// the row-pointer slot still holds n + 1 entries, the device copy of the row
// pointers of a host-resident matrix).  `sweep`: LZ_SWEEP_* request; the
// sweep-block copy is reserved when it applies (sweep_applies).
Plan make_plan(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t prec, bool relabel = true,
               int sweep = -1);
// Whether a relabelled matrix of this size gets the sweep-block copy:
// request 1 always (if the sort's 32-bit sizes reach), 0 never, -1 (auto)
// where its SpMV measured faster than the tile layouts.
bool sweep_applies(int64_t n, int64_t nnz, int prec, int request);
// Scratch bytes of the segmented sort of nnz entries in nb blocks (its own
// size query).
size_t sweep_sort_bytes(int64_t nnz, int64_t nb);

// Device pointers of a solve, resolved from a plan and a workspace base.
struct Bufs {
    State* st;
    void* V;
    void* w;
    double* part;      // per-workgroup partials: max(g_dense, 1024) * 256 doubles
    double* part2;     // second partial buffer (SpMV alpha, residual)
    uint64_t* scan;    // scan scratch (degree-class histogram)
    uint64_t* bsum;    // scan block sums
    double* Y;         // Ritz vectors, row-major n x K, before normalisation
    double* Z;         // A Y, row-major n x K (residual check)
    double* gram;      // Gram partials (GRAM_PARTS x 64 x 64), then the reduced 64 x 64
    int32_t* ob;       // SpMV tiles: first owned row of every tile (n_tiles + 1)
    uint32_t* tk;      // split-row tickets, one per owner tile
    double* head;      // split-row pieces at the start of a tile (n_tiles x KB2)
    double* tail;      // split-row pieces at the end of a tile (n_tiles x KB2)
    int64_t* rp2;      // hub-first relabelled CSR
    int32_t* col2;
    void* val2;
    int32_t* perm;
    int32_t* iperm;
    double* gm;        // Gram matrix of the unit stored basis, NCMAX x NCMAX
    // Sweep-block copy (Plan.sweep): first owned row and first entry of
    // every block (nb + 1), the entries' columns, rows within the block and
    // values in column order; the sort's payload in row order (swvin) and in
    // column order (swsrc), and its scratch.
    int32_t* swob;
    int64_t* swe;
    int32_t* swcol;
    uint16_t* swrl;
    void* swval;
    uint32_t* swsrc;
    uint32_t* swvin;
    void* swtmp;
    uint32_t* swq;     // per-XCD work counters of the sweep fill (8), zeroed by the block-table kernel
};
Bufs resolve(const Plan& p, void* base);

// Matrix pointers.
struct Csr {
    const int64_t* rowptr;
    const int32_t* col;
    const void* val;
    int64_t n, nnz;
};

// ------------------------------------------------------------- launchers
hipError_t launch_setup(const Plan& p, const Bufs& b, const Csr& a, uint64_t seed, int reorth, int reorder,
                        hipStream_t s);
hipError_t launch_init(const Plan& p, const Bufs& b, hipStream_t s);
// One Lanczos iteration (SpMV or restart draw, reorthogonalisation, store);
// `reorth` is the solve's LZ_REORTH_* mode (it selects the kernels).
// `ncols_bound` >= j+1 for every j the iteration can see.
// With `ev` non-null, ev[0] is recorded before the SpMV and ev[1] after it.
hipError_t launch_iteration(const Plan& p, const Bufs& b, const Csr& a, int ncols_bound, int reorth,
                            hipStream_t s, hipEvent_t* ev = nullptr);
// The Lanczos-step SpMV of the current iteration (or its restart draw).
hipError_t launch_spmv_step(const Plan& p, const Bufs& b, const Csr& a, hipStream_t s);
// Column checks 0 <= col[e] < n of entries [e0, e1) (col indexed by matrix
// entry); a failure sets the solve status to LZ_ERR_INVALID_ARG.
void launch_validate_cols(State* st, const int32_t* col, int64_t e0, int64_t e1, int64_t n, hipStream_t s);
// The LDS copy of the head of x pays off for relabelled (power-law)
// matrices in the mixed modes and costs occupancy elsewhere.  Measured on
// MI355X: R-MAT scale 23 FP32 1.79 -> 1.59 ms, BF16 1.63 -> 1.25 ms; scale
// 20 BF16 90 -> 80 us but FP32 102 -> 105 us; banded FP32 0.77 -> 1.15 ms.
inline bool want_xcache(const Plan& p, bool relabelled) {
    if (!relabelled) return false;
    if (p.prec == 2) return p.n >= (int64_t(1) << 20);
    if (p.prec == 1) return p.n >= (int64_t(1) << 22);
    return false;
}
// The relabelling decision of the setup kernels, for callers that hold the
// row pointer on the host (same integer test as on the device).
bool host_relabel_decision(const int64_t* rowptr_host, int64_t n, int64_t nnz, int reorder);
// The sweep-block copy of the relabelled matrix, in two parts around the
// relabelling fill (which writes the sort payload): the block table, then the
// segmented sort and the fill of rows and values.  Kernels return unless the
// device chose PACK_SWEEP (the sort then sees empty blocks).
void launch_sweep_blocks(const Plan& p, const Bufs& b, hipStream_t s);
hipError_t launch_sweep_sort(const Plan& p, const Bufs& b, hipStream_t s);
hipError_t launch_finish(const Plan& p, const Bufs& b, const Csr& a, double* out_vals,
                         double* out_vecs, int report, hipStream_t s);
// Copies the state into a device-resident lz_report (stream-ordered calls).
// `xcache_if_relabelled`: the SpMV staged the head of x in LDS whenever the
// device chose the hub-first order.
hipError_t launch_report(const Plan& p, const Bufs& b, void* d_report, int xcache_if_relabelled, hipStream_t s);
hipError_t launch_spmv_plain(const Plan& p, const Bufs& b, const Csr& a, const void* x, void* y,
                             hipStream_t s);
hipError_t launch_jacobi_only(const double* alpha, const double* offdiag, int m, State* st,
                              hipStream_t s);
// max |X^T X - I| of the first st->j columns of X (scales st->scale) into
// st->ortho_loss, with the kernels of the solve report.
hipError_t launch_gram_only(int prec, const void* X, int64_t ldx, int64_t n, State* st, double* gram,
                            hipStream_t s);

}  // namespace lz
