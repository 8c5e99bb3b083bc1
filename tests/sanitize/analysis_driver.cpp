// Host-only driver of the library's analysis (analysis.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py: reads a CSR system from a binary file
// (int64 n, int64 nnz, double tau, int32 ordering, int32 tile_kib; then rowptr, colidx, values),
// runs the analysis and prints its sizes as one line of key=value pairs, or the status and the
// message of a rejected input.  Any sanitizer report makes the process exit non-zero.
//
// It also replays both triangular-solve schedules on the CPU the way the solve kernel reads
// them (tiles in hand-out order; a staged tile's rows and externals in LDS slots, its entries
// referring to slots; unstaged one-row tiles reading global rows; dense segments as a block
// pass over references outside the segment, then a column sweep over the column-major
// strictly lower block) with random factor values, starting from a solution vector of NaN, and
// compares the result with plain substitution over the triangle's CSR (sched_l / sched_u =
// the relative difference, or the first violated property).  A reference to a value that is
// not final yet, a wrong slot or block index, a row solved twice or never, a segment whose
// rows do not fit its lanes, or a tile over its LDS budget all show up there.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2401_13926_amd/csrc/analysis.hpp"

namespace {

// rp/ci: the strict triangle's rows in pivot-step space (L: columns < row, U: columns > row);
// lower: L (unit diagonal) or U (diagonal d).  Returns "ok=<max relative difference>" or an error.
std::string replay(const kkt::TriSchedule &sc, int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                   bool lower, int64_t tile_lds, int threads) {
    std::mt19937_64 gen(lower ? 11 : 12);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    std::vector<double> val(ci.size()), b(n), d(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) val[p] = 0.5 * uni(gen) / (double)(len ? len : 1);
        b[i] = uni(gen);
        d[i] = 1.5 + 0.5 * uni(gen);
    }
    // reference: plain substitution in the order the dependencies allow
    std::vector<double> ref(n);
    if (lower) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc += val[p] * ref[ci[p]];
            ref[i] = b[i] - acc;
        }
    } else {
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc += val[p] * ref[ci[p]];
            ref[i] = (b[i] - acc) / d[i];
        }
    }
    // the triangle's values as the refactorization leaves them: packed entries, then dense blocks
    if ((int64_t)sc.csr2ent.size() != (int64_t)ci.size()) return "csr2ent_size";
    std::vector<double> tv(sc.values(), 0.0);
    std::vector<int> hit(sc.values(), 0);
    for (size_t p = 0; p < ci.size(); ++p) {
        const int64_t e = sc.csr2ent[p];
        if (e < 0 || e >= sc.values() || hit[e]++) return "csr2ent_slot";
        tv[e] = val[p];
    }
    if ((int64_t)sc.rows.size() != n || (int64_t)sc.row_ent.size() != n + 1) return "rows_size";
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> out(n, nan);
    std::vector<int> solved(n, 0);
    for (int64_t t = 0; t < sc.tiles(); ++t) {
        const int32_t s0 = sc.tile_seg[t], s1 = sc.tile_seg[t + 1];
        const int32_t rb = sc.seg_row[s0], re = sc.seg_row[s1];
        const int32_t nr = re - rb;
        const int64_t eb = sc.row_ent[rb], ne = sc.row_ent[re] - eb;
        const int32_t xb = sc.tile_ext[t], nx = sc.tile_ext[t + 1] - xb;
        const int64_t db = sc.tile_dense[t], nd = sc.tile_dense[t + 1] - db;
        auto finish = [&](int32_t r, double res) -> bool {
            const int32_t i = sc.rows[r];
            if (i < 0 || i >= n || solved[i]++) return false;
            out[i] = res;
            return true;
        };
        if (!sc.tile_lds[t]) {  // one row, entries and sources in global memory
            if (nr != 1 || nd != 0 || nx != 0) return "unstaged_shape";
            double acc = 0.0;
            for (int64_t e = 0; e < ne; ++e) {
                const int32_t c = sc.ent_ref[eb + e];
                if (c < 0 || c >= n || std::isnan(out[c])) return "unstaged_ref";
                acc += tv[eb + e] * out[c];
            }
            const int32_t i = sc.rows[rb];
            if (!finish(rb, lower ? b[i] - acc : (b[i] - acc) / d[i])) return "row_twice";
            continue;
        }
        if (kkt::tile_lds_bytes(nr, nx, ne, nd) > tile_lds) return "tile_budget";
        // LDS: the tile's rows, then its externals (final before the tile starts)
        std::vector<double> xs(nr + nx, nan);
        for (int32_t k = 0; k < nx; ++k) {
            const int32_t c = sc.ext_src[xb + k];
            if (c < 0 || c >= n || std::isnan(out[c])) return "external_not_final";
            xs[nr + k] = out[c];
        }
        for (int64_t e = 0; e < ne; ++e)
            if (sc.ent_ref[eb + e] < 0 || sc.ent_ref[eb + e] >= nr + nx || sc.ent_ref[eb + e] > 0xFFFF) return "slot_range";
        auto row_sum = [&](int32_t r, double &acc) -> bool {  // r local
            acc = 0.0;
            for (int64_t e = sc.row_ent[rb + r] - eb; e < sc.row_ent[rb + r + 1] - eb; ++e) {
                const double x = xs[sc.ent_ref[eb + e]];
                if (std::isnan(x)) return false;
                acc += tv[eb + e] * x;
            }
            return true;
        };
        for (int32_t g = s0; g < s1; ++g) {
            const int32_t lb = sc.seg_row[g] - rb, le = sc.seg_row[g + 1] - rb, m = le - lb;
            const int32_t code = sc.seg_lg[g], lg = code & 0xF;
            if (m <= 0) return "empty_segment";
            if (((int64_t)m << lg) > ((code & kkt::kSegWave) ? 64 : threads)) return "segment_lanes";
            if (code & kkt::kSegDense) {
                if (m > kkt::kDenseRows || sc.seg_dofs[g] < 0 || sc.seg_dofs[g] + kkt::dense_block_values(m) > nd)
                    return "dense_block";
                std::vector<double> y(m);
                for (int32_t l = 0; l < m; ++l) {
                    double acc;
                    if (!row_sum(lb + l, acc)) return "dense_ref_not_final";
                    y[l] = b[sc.rows[rb + lb + l]] - acc;
                }
                const double *D = tv.data() + db + sc.seg_dofs[g];
                for (int32_t c = 0; c < m; ++c) {
                    const double xc = lower ? y[c] : y[c] / d[sc.rows[rb + lb + c]];
                    for (int32_t l = c + 1; l < m; ++l) y[l] -= D[(int64_t)c * m - (int64_t)c * (c + 1) / 2 + (l - c - 1)] * xc;
                }
                for (int32_t l = 0; l < m; ++l) {
                    const double res = lower ? y[l] : y[l] / d[sc.rows[rb + lb + l]];
                    xs[lb + l] = res;
                    if (!finish(rb + lb + l, res)) return "row_twice";
                }
                continue;
            }
            std::vector<double> res(m);
            for (int32_t l = 0; l < m; ++l) {  // rows of a segment are independent of each other
                double acc;
                if (!row_sum(lb + l, acc)) return "ref_not_final";
                const int32_t i = sc.rows[rb + lb + l];
                res[l] = lower ? b[i] - acc : (b[i] - acc) / d[i];
            }
            for (int32_t l = 0; l < m; ++l) {
                xs[lb + l] = res[l];
                if (!finish(rb + lb + l, res[l])) return "row_twice";
            }
        }
    }
    double scale = 0.0, diff = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!solved[i]) return "row_never_solved";
        scale = std::fmax(scale, std::fabs(ref[i]));
        diff = std::fmax(diff, std::fabs(out[i] - ref[i]));
    }
    char buf[64];
    std::snprintf(buf, sizeof buf, "ok:%.3e", scale > 0.0 ? diff / scale : diff);
    return buf;
}

// Replays the refactorization of another system with the same pattern from the hand-out
// metadata, as the refactorization kernel reads it: K's values in the vector-order copy (ksrc),
// items in hand-out order, each column staged through fsrc_k, its flat update list (relsrc,
// relpos, relslot) applied in order, the pivot guard (unit roundoff 2^-53 times the staged
// column's largest magnitude), L published to Ld (NaN until then: a source read before it is
// final means an item depends on a later one, which the kernel's progress argument forbids),
// and every value scattered into the solve layout through f2t.  lx/ux come back from the solve
// layout in exchange layout, as kkt_get_factor_values reads them.
std::string replay_refactor(const kkt::Analysis &a, const std::vector<double> &vals, std::vector<double> &lx,
                            std::vector<double> &ux) {
    if (!a.phys) return "no_flat_list";
    const int64_t f = a.nnz_f();
    std::vector<double> kval(a.ksrc.size());
    for (size_t t = 0; t < kval.size(); ++t) kval[t] = vals[a.ksrc[t]];
    std::vector<double> ld(f, std::numeric_limits<double>::quiet_NaN()), tv(a.t_size, 0.0);
    std::vector<int> written(a.t_size, 0);
    for (size_t it = 0; it + 1 < a.ref_item.size(); ++it) {
        for (int64_t p = a.ref_item[it]; p < a.ref_item[it + 1]; ++p) {
            const int64_t c0 = a.pc[p], len = a.pc[p + 1] - c0;
            const int32_t nu = a.pnu[p];
            if (len <= 0 || nu < 0 || nu >= len) return "column_shape";
            std::vector<double> x(len);
            double cm = 0.0;
            for (int64_t e = 0; e < len; ++e) {
                const int64_t src = a.fsrc_k[c0 + e];
                x[e] = src >= 0 ? kval[src] : 0.0;
                cm = std::fmax(cm, std::fabs(x[e]));
            }
            for (int64_t b = a.pu[p]; b < a.pu[p + 1]; ++b) {
                const int64_t src = a.relsrc[b];
                const int32_t pos = a.relpos[b], slot = a.relslot[b];
                if (src < 0 || src >= f || pos <= 0 || pos >= len || slot < 0 || slot >= nu) return "update_index";
                const double l = ld[src];
                if (std::isnan(l)) return "source_not_final";
                const double prod = l * x[slot];
                x[pos] = x[pos] - prod;
            }
            double d = x[nu];
            const double ur = 0x1p-53, cmx = cm > 0.0 ? cm : 1.0;
            if (!(std::fabs(d) > ur * cmx) || !std::isfinite(d)) d = (d < 0.0 ? -1.0 : 1.0) * ur * cmx;
            for (int64_t e = 0; e < len; ++e) {
                double v = x[e];
                if (e == nu) v = d;
                else if (e > nu) v = v / d;
                if (e > nu) ld[c0 + e] = v;
                const int64_t t = a.f2t[c0 + e];
                if (t < 0 || t >= a.t_size || written[t]++) return "f2t_slot";
                tv[t] = v;
            }
        }
    }
    lx.resize(a.nnz_l());
    ux.resize(a.nnz_u());
    for (int64_t q = 0; q < a.nnz_l(); ++q) lx[q] = tv[a.f2t[a.l2f[q]]];
    for (int64_t q = 0; q < a.nnz_u(); ++q) ux[q] = tv[a.f2t[a.u2f[q]]];
    return "ok";
}

}  // namespace

int main(int argc, char **argv) {
    // input.bin may end with a second system's values (nnz float64): then the refactorization
    // is replayed with them and the factors written to factors.bin (float64 lx, then ux)
    if (argc != 2 && argc != 3) {
        std::fprintf(stderr, "usage: %s input.bin [factors.bin]\n", argv[0]);
        return 2;
    }
    std::FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0, nnz = 0;
    double tau = 0.0;
    int32_t ordering = 0, tile_kib = 0;
    bool ok = std::fread(&n, 8, 1, f) == 1 && std::fread(&nnz, 8, 1, f) == 1 && std::fread(&tau, 8, 1, f) == 1 &&
              std::fread(&ordering, 4, 1, f) == 1 && std::fread(&tile_kib, 4, 1, f) == 1;
    std::vector<int64_t> rp(ok ? n + 1 : 0);
    std::vector<int32_t> ci(ok ? nnz : 0);
    std::vector<double> v(ok ? nnz : 0);
    ok = ok && std::fread(rp.data(), 8, rp.size(), f) == rp.size() && std::fread(ci.data(), 4, ci.size(), f) == ci.size() &&
         std::fread(v.data(), 8, v.size(), f) == v.size();
    std::vector<double> v2(ok ? nnz : 0);
    const bool second = ok && argc == 3 && std::fread(v2.data(), 8, v2.size(), f) == v2.size();
    std::fclose(f);
    if (!ok) return 2;
    kkt::AnalysisOptions opt;
    opt.ordering = ordering;
    opt.pivot_tau = tau;
    opt.tile_threads = 256;
    opt.tile_rows = 2048;
    opt.tile_lds = tile_kib > 0 ? tile_kib * 1024 : 32768;  // the library default
    opt.dense_reserve_l = opt.tile_lds / 2;
    opt.narrow_columns = 1024;
    kkt::Analysis a;
    std::string msg;
    const int rc = kkt::analyze(opt, n, rp.data(), ci.data(), v.data(), a, &msg);
    if (rc != kkt::AN_OK) {
        std::printf("status=%d message=%s\n", rc, msg.c_str());
        return 0;
    }
    int64_t offdiag = 0;
    for (int64_t k = 0; k < n; ++k) offdiag += a.prow[k] != a.q[k];
    const std::string sl = replay(a.lsched, n, a.lrp, a.lci, true, opt.tile_lds, opt.tile_threads);
    const std::string su = replay(a.usched, n, a.urp, a.uci, false, opt.tile_lds, opt.tile_threads);
    int64_t dense_l = 0;
    for (int32_t code : a.lsched.seg_lg) dense_l += (code & kkt::kSegDense) != 0;
    std::printf("status=0 nnz_l=%lld nnz_u=%lld levels_refactor=%lld levels_l=%lld levels_u=%lld updates=%lld "
                "offdiag_pivots=%lld tiles_l=%lld tiles_u=%lld items=%lld dense_l=%lld sched_l=%s sched_u=%s\n",
                (long long)a.nnz_l(), (long long)a.nnz_u(), (long long)a.levels_refactor, (long long)a.lsched.levels,
                (long long)a.usched.levels, (long long)a.updates(), (long long)offdiag, (long long)a.lsched.tiles(),
                (long long)a.usched.tiles(), (long long)a.ref_item.size() - 1, (long long)dense_l, sl.c_str(), su.c_str());
    if (second) {
        std::vector<double> lx, ux;
        const std::string r = replay_refactor(a, v2, lx, ux);
        std::printf("refactor=%s\n", r.c_str());
        if (r == "ok") {
            std::FILE *o = std::fopen(argv[2], "wb");
            if (!o) return 2;
            const bool w = std::fwrite(lx.data(), 8, lx.size(), o) == lx.size() &&
                           std::fwrite(ux.data(), 8, ux.size(), o) == ux.size();
            std::fclose(o);
            if (!w) return 2;
        }
    }
    return 0;
}
