// Host-only driver of the library's analysis (analysis.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py: reads a CSR system from a binary file
// (int64 n, int64 nnz, double tau, int32 ordering, int32 tile_kib; then rowptr, colidx, values),
// runs the analysis and prints its sizes as one line of key=value pairs, or the status and the
// message of a rejected input.  Any sanitizer report makes the process exit non-zero.
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "../../paper_2401_13926_amd/csrc/analysis.hpp"

int main(int argc, char **argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s input.bin\n", argv[0]);
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
    std::printf("status=0 nnz_l=%lld nnz_u=%lld levels_refactor=%lld levels_l=%lld levels_u=%lld updates=%lld "
                "offdiag_pivots=%lld tiles_l=%lld tiles_u=%lld items=%lld\n",
                (long long)a.nnz_l(), (long long)a.nnz_u(), (long long)a.levels_refactor, (long long)a.lsched.levels,
                (long long)a.usched.levels, (long long)a.updates(), (long long)offdiag, (long long)a.lsched.tiles(),
                (long long)a.usched.tiles(), (long long)a.ref_item.size() - 1);
    return 0;
}
