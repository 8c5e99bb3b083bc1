// Host-side analysis for the KKT refactorization solver: ordering, pivoted LU of the first
// system, and every schedule / layout the GPU kernels consume.  Pure C++, no HIP calls.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace kkt {

enum { ORDER_MD = 0, ORDER_ND = 1 };

// Refactorization hand-out: columns of at most kLaneLen entries run one per lane of a
// wavefront (64 x kLaneLen entries fill its LDS stage of 1,024); longer columns of a wide
// level are handed out kLaneChunk at a time.
constexpr int kLaneLen = 16;
constexpr int kLaneChunk = 8;

struct AnalysisOptions {
    int ordering = ORDER_MD;     // exact minimum degree, or BFS nested dissection
    const int32_t *fixed_order = nullptr;  // when set: this column order (n entries) is used
    int64_t nd_leaf = 64;
    double pivot_tau = 1e-10;
    int tile_threads = 256;      // threads of a triangular-solve block
    int tile_rows = 2048;        // rows of a tile at most
    int64_t tile_lds = 32768;    // LDS bytes of a staged tile at most (tile_lds_bytes)
    // LDS that tiles keep free for dense blocks (0: no dense segments), per triangle.  The top
    // of L's DAG is many levels of few long rows, where fusing pays; measured on the 60k
    // sequence, fusing in U (shorter rows, wider levels) cost more than it saved.
    int64_t dense_reserve_l = 16384;
    int64_t dense_reserve_u = 0;
    int narrow_columns = 1024;   // refactorization levels with at most this many columns are
                                 // handed out one column at a time
};

// Flags in TriSchedule::seg_lg: the segment's rows fit one wavefront; the segment is a
// *dense* one (several consecutive levels, at most kDenseRows rows, whose references to each
// other are kept as a dense strictly lower triangle in solve order and resolved by a
// wavefront-level column sweep; the packed entries of its rows hold only the references to
// earlier segments and tiles).
constexpr int32_t kSegWave = 0x40;
constexpr int32_t kSegDense = 0x80;
constexpr int kDenseRows = 64;
// A solve window whose first level has at most this many rows keeps part of its tile budget
// for dense blocks (the narrow top of the DAG); wider windows use the whole budget.
constexpr int kDenseWindowRows = 2048;

// Schedule of one triangular solve.  A tile is a contiguous run of rows solved by one block;
// it is cut into segments, each a set of mutually independent rows covered by one pass of the
// block (2^lg lanes per row), with a block barrier between segments.  Tiles are handed out in
// order; every reference of a row is to an earlier tile or an earlier segment of its own tile.
//
// Entries are stored "packed": the rows of the solve order one after the other, each row's
// entries in ascending column order.  A staged tile (tile_lds = 1) is copied into LDS when its
// block takes it: its entries, its rows' right-hand-side data, and the solution values of the
// rows it references in earlier tiles ("externals"); its references are then LDS slots
// (0..rows-1: the tile's own rows, rows + k: external k).  An unstaged tile (one row too long
// to stage) reads its entries from global memory and its references are source rows.
struct TriSchedule {
    std::vector<int32_t> rows;      // solve order
    std::vector<int32_t> tile_seg;  // first segment of each tile (tiles + 1)
    std::vector<int32_t> seg_row;   // start of each segment in rows (segments + 1)
    std::vector<int32_t> seg_lg;    // log2 of the lanes per row of each segment, | kSegWave when
                                    // the segment fits one wavefront (solved by wavefront 0)
    std::vector<int64_t> row_ent;   // first packed entry of each position of rows (n + 1)
    std::vector<int32_t> ent_ref;   // per packed entry: LDS slot (staged tile) or source row
    std::vector<int32_t> tile_ext;  // first external of each tile (tiles + 1)
    std::vector<int32_t> ext_src;   // source row of each external
    std::vector<uint8_t> tile_lds;  // 1: staged in LDS, 0: entries read from global memory
    std::vector<int64_t> csr2ent;   // CSR entry (row-wise layout of the triangle) -> index in the
                                    // triangle's values: [packed entries | dense blocks]
    std::vector<int64_t> tile_dense;  // first dense-block value of each tile (tiles + 1), index in
                                      // the triangle's values
    std::vector<int32_t> seg_dofs;  // dense segment: offset of its block within the tile's dense
                                    // values (column-major strictly lower triangle), else -1
    int64_t packed = 0;             // number of packed entries
    int64_t values() const { return tile_dense.empty() ? packed : tile_dense.back(); }
    int64_t levels = 0;             // depth of the dependency DAG
    int64_t windows = 0;            // groups of levels whose tiles are mutually independent
    int64_t tiles() const { return (int64_t)tile_seg.size() - 1; }
    int64_t segments() const { return (int64_t)seg_row.size() - 1; }
};

// LDS bytes a staged tile needs with FP64 values (the kernel's layout: solution slots, rhs,
// diagonal, entry values, dense-block values; row ids, column-permutation ids, row offsets;
// 16-bit references).
inline int64_t tile_lds_bytes(int64_t rows, int64_t ext, int64_t ent, int64_t dense = 0) {
    return 8 * (rows + ext) + 36 * rows + 10 * ent + 8 * dense + 32;
}
inline int64_t dense_block_values(int64_t m) { return m * (m - 1) / 2; }

// Everything derived from the pattern and the first system's values.
//
// Index spaces: "original" rows/columns are those of K; "steps" are pivot steps of the
// factorization P K Q = L U (row k of P K Q is original row prow[k], column k is q[k]).
struct Analysis {
    int64_t n = 0, nnz = 0;
    std::vector<int64_t> rowptr;  // K pattern (copy), CSR
    std::vector<int32_t> colidx;

    std::vector<int32_t> q, prow, pinv;
    int64_t offdiag_pivots = 0;

    // Factors in "exchange" layout (matches kkt_get_factor_pattern):
    //   L: strictly lower, per column original rows ascending; U: per column steps ascending,
    //   diagonal last.  Values of system 1 from the pivoted factorization.
    std::vector<int64_t> lp, up;
    std::vector<int32_t> li, ui;
    std::vector<double> lx, ux;

    // Combined factor F = L + U in step space, column-compressed, rows ascending:
    // column j = U part (rows < j), diagonal (row j), L part (rows > j).
    std::vector<int64_t> fp;      // n+1
    std::vector<int32_t> fi;      // f
    std::vector<int32_t> fdiag;   // per column: offset of the diagonal inside the column
    std::vector<int64_t> fsrc;    // per F entry: index into K's CSR values, or -1 (fill)
    std::vector<double> fx;       // system-1 values in F layout (host reference)

    // Update positions: for column j, for each U-part row k ascending, for each L-part
    // entry of column k in order: offset (inside column j) of that row.
    std::vector<int64_t> relptr;  // n+1
    std::vector<int32_t> relpos;  // sum of updates
    // The same updates as a flat list (the refactorization's paths when it exists): the F
    // index of the L entry each update applies, and the position in column j of its source's
    // U entry.  Empty when the factor has 2^31 entries or more.
    std::vector<int32_t> relsrc;
    std::vector<int32_t> relslot;

    // Refactorization schedule: columns sorted by (DAG level, index).
    std::vector<int32_t> col_order;
    std::vector<int32_t> col_level;  // DAG level of each col_order position (non-decreasing)
    int64_t levels_refactor = 0;
    // Hand-out items of the refactorization, in col_order (level) order: item t covers
    // positions [ref_item[t], ref_item[t + 1]).  In a wide level (more than narrow_columns
    // columns) a lane item holds up to 64 columns with at most kLaneLen entries each,
    // refactored one per lane, and the longer columns go kLaneChunk per item; in a narrow
    // level (the dependency chain at the top of the elimination tree) every column is an item
    // of its own, refactored by a whole wavefront.  Within a level, col_order puts the
    // lane-sized columns first.
    std::vector<int32_t> ref_item;
    std::vector<uint8_t> ref_item_lane;

    // Row-wise triangles in step space (strict L, strict U), from which the solve schedules
    // are built.  Solve layout T = [L values | strict U values | U diagonal (n, step order)],
    // each triangle's values being its schedule's [packed entries | dense blocks]; f2t maps
    // each F entry to its T index.
    std::vector<int64_t> lrp, urp;  // n+1 each
    std::vector<int32_t> lci, uci;  // column indices (steps), ascending per row
    std::vector<int32_t> f2t;
    int64_t t_size = 0;  // values in T (dense blocks include explicit zeros)

    // Triangular-solve schedules (L forward, U backward).
    TriSchedule lsched, usched;

    // Exchange layout -> F position (for copying device values back).
    std::vector<int64_t> l2f, u2f;

    // Order of the vectors inside a solve (the Krylov basis, residuals, iterates): position k
    // holds original index vperm[k], a reverse Cuthill-McKee order of K + K^T, so that the rows
    // one block of the matrix-vector products handles reference nearby entries.  The Krylov
    // kernels' copy of K is in that order: row k is original row vperm[k], its entries in their
    // original order with columns renumbered by vpinv (each row's terms are still summed in
    // ascending original column), ksrc the original CSR position of each entry.  fsrc_k is
    // fsrc in terms of that copy; prow_k, q_k are prow and q renumbered by vpinv.
    std::vector<int32_t> vperm, vpinv;
    std::vector<int64_t> krp;
    std::vector<int32_t> kci;
    std::vector<int64_t> ksrc, fsrc_k;
    std::vector<int32_t> prow_k, q_k;

    // Device layout with the flat list (phys): F's columns are stored in col_order, so the
    // columns of one hand-out item (the 64 of a lane item in particular) are side by side, and
    // the update lists follow the same order.  pc[p] / pu[p] (n + 1 each, ascending) are the
    // first F position / first update of the column at col_order position p, pnu[p] its
    // diagonal offset.  relpos, relsrc and relslot are then in that order, and relsrc, f2t,
    // fsrc_k, l2f and u2f hold these F positions.  Without the flat list F keeps the column
    // order of fp.
    bool phys = false;
    std::vector<int64_t> pc, pu;
    std::vector<int32_t> pnu;

    double seconds = 0.0;

    int64_t nnz_l() const { return (int64_t)li.size(); }
    int64_t nnz_u() const { return (int64_t)ui.size(); }
    int64_t nnz_f() const { return (int64_t)fi.size(); }
    int64_t updates() const { return (int64_t)relpos.size(); }
};

enum AnalysisStatus { AN_OK = 0, AN_EINVAL = 1, AN_ENOMEM = 2, AN_ESINGULAR = 3 };

// Runs the whole analysis.  On failure returns the status and sets *msg.
int analyze(const AnalysisOptions &opt, int64_t n, const int64_t *rowptr, const int32_t *colidx,
            const double *values, Analysis &out, std::string *msg);

// Exposed for tests of the orderings alone.
void vector_order(int64_t n, const int64_t *rowptr, const int32_t *colidx, std::vector<int32_t> &perm);
int nested_dissection(int64_t n, const int64_t *rowptr, const int32_t *colidx, int64_t leaf,
                      std::vector<int32_t> &q);

}  // namespace kkt
