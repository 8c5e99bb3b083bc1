// Host-side analysis for the KKT refactorization solver: ordering, pivoted LU of the first
// system, and every schedule / layout the GPU kernels consume.  Pure C++, no HIP calls.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace kkt {

enum { ORDER_MD = 0, ORDER_ND = 1 };

struct AnalysisOptions {
    int ordering = ORDER_MD;     // exact minimum degree, or BFS nested dissection
    int64_t nd_leaf = 64;
    double pivot_tau = 0.1;
    int tile_threads = 256;      // threads of a triangular-solve block
    int narrow_rows = 256;       // levels with at most this many rows join multi-level tiles
    int tile_rows = 2048;        // rows of a multi-level tile (its values live in LDS)
    int narrow_columns = 1024;   // refactorization levels with at most this many columns are
                                 // handed out one column at a time
};

// Schedule of one triangular solve.  Rows are sorted by DAG level.  A tile is a contiguous
// run of rows processed by one block: either a run of whole narrow levels (processed level
// by level with a block barrier in between, values kept in LDS) or a slice of one wide level.
struct TriSchedule {
    std::vector<int32_t> rows;      // solve order
    std::vector<int32_t> lev_ptr;   // start of each level in rows (levels + 1)
    std::vector<int8_t> lev_lg;     // log2 of the lanes per row of each level
    std::vector<int32_t> tile_row;  // start of each tile in rows (tiles + 1)
    std::vector<int32_t> tile_lev;  // level of each tile's first row
    std::vector<int32_t> ref;       // per CSR entry: source row (>= 0), or -(slot + 1) when the
                                    // source row is in the same tile (LDS slot)
    int64_t levels = 0;
    int64_t tiles() const { return (int64_t)tile_row.size() - 1; }
};

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

    // Refactorization schedule: columns sorted by (DAG level, index).
    std::vector<int32_t> col_order;
    int64_t levels_refactor = 0;
    // Columns at col_order positions >= refactor_split belong to narrow levels (few columns
    // each, mostly a dependency chain): they are handed out one at a time so that each starts
    // its update chain as early as possible.
    int64_t refactor_split = 0;

    // Solve layout T = [L strict CSR (nnz_l) | U strict CSR (nnz_u - n) | U diagonal (n)],
    // all in step space; f2t maps each F entry to its T index.
    std::vector<int64_t> lrp, urp;  // n+1 each
    std::vector<int32_t> lci, uci;  // column indices (steps), ascending per row
    std::vector<int32_t> f2t;

    // Triangular-solve schedules (L forward, U backward).
    TriSchedule lsched, usched;

    // Exchange layout -> F position (for copying device values back).
    std::vector<int64_t> l2f, u2f;

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

// Exposed for tests of the ordering alone.
int nested_dissection(int64_t n, const int64_t *rowptr, const int32_t *colidx, int64_t leaf,
                      std::vector<int32_t> &q);

}  // namespace kkt
