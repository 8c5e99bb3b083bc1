// Host analysis: nested-dissection ordering, threshold-pivoted left-looking sparse LU of the
// first system, and the GPU schedules.  Section 1.3 of the paper describes the strategy
// (symbolic analysis and pivoted factorization once on the host, numeric refactorization
// reusing the pivot sequence afterwards); the paper delegates this step to KLU without
// stating its settings, so the ordering and pivot rule here are a fixed, deterministic
// specification (described at each function) that any independent implementation
// reproduces bit for bit.
//
// Built with -ffp-contract=off: every product and difference in the factorization is
// rounded on its own, so the factor values are reproducible.
#include "analysis.hpp"

#include <algorithm>
#include <chrono>
#include <iterator>
#include <set>
#include <cmath>
#include <limits>
#include <new>

namespace kkt {
namespace {

bool csr_valid(int64_t n, const int64_t *rp, const int32_t *ci, std::string *msg) {
    if (n < 1) {
        *msg = "n must be >= 1";
        return false;
    }
    if (rp[0] != 0) {
        *msg = "rowptr[0] must be 0";
        return false;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) {
            *msg = "rowptr decreases at row " + std::to_string(i);
            return false;
        }
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) {
                *msg = "column index out of range in row " + std::to_string(i);
                return false;
            }
            if (p > rp[i] && ci[p] <= ci[p - 1]) {
                *msg = "columns not strictly ascending in row " + std::to_string(i);
                return false;
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------------------
// Nested dissection on the graph of A + A^T without its diagonal.
//
//   order(S): |S| <= leaf            -> S ascending
//             G[S] disconnected      -> order(component) for each component, components by
//                                       their smallest vertex
//             otherwise              -> root r: start at the vertex of least degree in G[S]
//                                       (ties: smallest), BFS, jump to the least-degree
//                                       vertex of the last level (ties: smallest) while the
//                                       eccentricity increases.  Levels L_0..L_e from r.
//                                       e < 2: S ascending.  Else the separator is L_s with
//                                       s the first level whose cumulative size reaches
//                                       |S|/2, clamped to [1, e-1]; emit order(L_<s),
//                                       order(L_>s), then L_s ascending.
// ---------------------------------------------------------------------------------------
class Dissector {
  public:
    Dissector(int64_t n, const int64_t *rp, const int32_t *ci, int64_t leaf) : n_(n), leaf_(leaf) {
        std::vector<int64_t> deg(n + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] != i) {
                    ++deg[i + 1];
                    ++deg[ci[p] + 1];
                }
        for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
        std::vector<int32_t> adj(deg[n]);
        std::vector<int64_t> pos(deg.begin(), deg.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] != i) {
                    adj[pos[i]++] = ci[p];
                    adj[pos[ci[p]]++] = (int32_t)i;
                }
        gptr_.assign(n + 1, 0);
        gadj_.reserve(adj.size());
        for (int64_t i = 0; i < n; ++i) {
            auto b = adj.begin() + deg[i], e = adj.begin() + deg[i + 1];
            std::sort(b, e);
            auto last = std::unique(b, e);
            gadj_.insert(gadj_.end(), b, last);
            gptr_[i + 1] = (int64_t)gadj_.size();
        }
        owner_.assign(n, 0);
        seen_.assign(n, 0);
        dist_.assign(n, 0);
        bfs_.resize(n);
    }

    void run(std::vector<int32_t> &q) {
        out_ = &q;
        q.clear();
        q.reserve(n_);
        std::vector<int32_t> all(n_);
        for (int64_t v = 0; v < n_; ++v) all[v] = (int32_t)v;
        order(all, 0);
    }

  private:
    int64_t n_, leaf_;
    std::vector<int64_t> gptr_;
    std::vector<int32_t> gadj_;
    std::vector<int32_t> owner_;  // set tag of each vertex
    std::vector<uint64_t> seen_;  // BFS visit tags
    uint64_t tick_ = 0;
    std::vector<int32_t> dist_, bfs_;
    int32_t next_tag_ = 1;
    std::vector<int32_t> *out_ = nullptr;

    int64_t degree_in(int32_t v, int32_t tag) const {
        int64_t d = 0;
        for (int64_t p = gptr_[v]; p < gptr_[v + 1]; ++p) d += owner_[gadj_[p]] == tag;
        return d;
    }

    // BFS from root restricted to `tag`; bfs_[0..count) in visit order, dist_ set.
    int32_t bfs(int32_t root, int32_t tag, int64_t &count) {
        const uint64_t t = ++tick_;
        int64_t head = 0, tail = 0;
        bfs_[tail++] = root;
        seen_[root] = t;
        dist_[root] = 0;
        int32_t ecc = 0;
        while (head < tail) {
            const int32_t v = bfs_[head++];
            for (int64_t p = gptr_[v]; p < gptr_[v + 1]; ++p) {
                const int32_t u = gadj_[p];
                if (owner_[u] != tag || seen_[u] == t) continue;
                seen_[u] = t;
                dist_[u] = dist_[v] + 1;
                ecc = std::max(ecc, dist_[u]);
                bfs_[tail++] = u;
            }
        }
        count = tail;
        return ecc;
    }

    void emit_ascending(std::vector<int32_t> &s) {
        std::sort(s.begin(), s.end());
        out_->insert(out_->end(), s.begin(), s.end());
    }

    void order(std::vector<int32_t> &s, int32_t tag) {
        const int64_t size = (int64_t)s.size();
        if (size <= leaf_) {
            emit_ascending(s);
            return;
        }
        std::sort(s.begin(), s.end());
        int64_t reached = 0;
        bfs(s[0], tag, reached);
        if (reached < size) {
            // components, each collected from its smallest unvisited vertex
            const uint64_t t = ++tick_;
            std::vector<std::vector<int32_t>> comps;
            for (int32_t v0 : s) {
                if (seen_[v0] == t) continue;
                std::vector<int32_t> comp{v0};
                seen_[v0] = t;
                for (size_t h = 0; h < comp.size(); ++h) {
                    const int32_t v = comp[h];
                    for (int64_t p = gptr_[v]; p < gptr_[v + 1]; ++p) {
                        const int32_t u = gadj_[p];
                        if (owner_[u] == tag && seen_[u] != t) {
                            seen_[u] = t;
                            comp.push_back(u);
                        }
                    }
                }
                comps.push_back(std::move(comp));
            }
            for (auto &c : comps) {
                const int32_t ctag = next_tag_++;
                for (int32_t v : c) owner_[v] = ctag;
                order(c, ctag);
            }
            return;
        }
        int32_t root = s[0];
        int64_t best = std::numeric_limits<int64_t>::max();
        for (int32_t v : s) {  // ascending: first strict minimum is the smallest index
            const int64_t d = degree_in(v, tag);
            if (d < best) {
                best = d;
                root = v;
            }
        }
        int64_t count = 0;
        int32_t ecc = bfs(root, tag, count);
        while (true) {
            int32_t cand = -1;
            int64_t cd = std::numeric_limits<int64_t>::max();
            for (int64_t t = 0; t < count; ++t) {
                const int32_t v = bfs_[t];
                if (dist_[v] != ecc) continue;
                const int64_t d = degree_in(v, tag);
                if (d < cd || (d == cd && v < cand)) {
                    cd = d;
                    cand = v;
                }
            }
            int64_t c2 = 0;
            const int32_t e2 = bfs(cand, tag, c2);
            if (e2 <= ecc) break;
            root = cand;
            ecc = e2;
            count = c2;
        }
        ecc = bfs(root, tag, count);
        if (ecc < 2) {
            emit_ascending(s);
            return;
        }
        std::vector<int64_t> width(ecc + 1, 0);
        for (int32_t v : s) ++width[dist_[v]];
        int32_t sep = 0;
        int64_t cum = 0;
        for (int32_t l = 0; l <= ecc; ++l) {
            cum += width[l];
            if (2 * cum >= size) {
                sep = l;
                break;
            }
        }
        sep = std::min(std::max(sep, 1), ecc - 1);
        std::vector<int32_t> below, above, middle;
        for (int32_t v : s) {
            if (dist_[v] < sep) below.push_back(v);
            else if (dist_[v] > sep) above.push_back(v);
            else middle.push_back(v);
        }
        const int32_t tb = next_tag_++, ta = next_tag_++, tm = next_tag_++;
        for (int32_t v : below) owner_[v] = tb;
        for (int32_t v : above) owner_[v] = ta;
        for (int32_t v : middle) owner_[v] = tm;
        std::vector<int32_t>().swap(s);  // release the caller's copy before recursing
        order(below, tb);
        order(above, ta);
        emit_ascending(middle);
    }
};

// ---------------------------------------------------------------------------------------
// Reverse Cuthill-McKee order of the graph of A + A^T without its diagonal (the order of the
// vectors inside a solve; it only decides where the matrix-vector products find their
// operands, never an operation or its order).  Components by their smallest vertex; in each,
// the start is pseudo-peripheral (least degree in the component, ties: smallest index, then
// the least-degree vertex of the last BFS level, ties: smallest, while the eccentricity
// grows); BFS visits the unvisited neighbours of a vertex by ascending (degree, index); the
// concatenated order is reversed.  perm[k] = vertex at position k.
// ---------------------------------------------------------------------------------------
void rcm_order(int64_t n, const int64_t *rp, const int32_t *ci, std::vector<int32_t> &perm) {
    std::vector<int64_t> gp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                ++gp[i + 1];
                ++gp[ci[p] + 1];
            }
    for (int64_t i = 0; i < n; ++i) gp[i + 1] += gp[i];
    std::vector<int32_t> gi(gp[n]);
    {
        std::vector<int64_t> w(gp.begin(), gp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (ci[p] != i) {
                    gi[w[i]++] = ci[p];
                    gi[w[ci[p]]++] = (int32_t)i;
                }
    }
    // sorted, duplicates (entries present in both triangles) removed
    std::vector<int64_t> deg(n);
    {
        int64_t out = 0, beg = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t end = gp[i + 1];
            std::sort(gi.begin() + beg, gi.begin() + end);
            const int64_t start = out;
            for (int64_t p = beg; p < end; ++p)
                if (p == beg || gi[p] != gi[p - 1]) gi[out++] = gi[p];
            gp[i] = start;
            beg = end;
            deg[i] = out - start;
        }
        gp[n] = out;
        gi.resize(out);
    }
    std::vector<int32_t> level(n, -1), comp;
    std::vector<uint8_t> done(n, 0);
    // BFS levels from r inside the component (level[] reset for `comp` afterwards); returns the
    // eccentricity and leaves the last level's least-(degree, index) vertex in *far
    auto bfs = [&](int32_t r, int32_t *far) {
        std::vector<int32_t> q{r};
        level[r] = 0;
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t v = q[h];
            for (int64_t p = gp[v]; p < gp[v + 1]; ++p)
                if (level[gi[p]] < 0) {
                    level[gi[p]] = level[v] + 1;
                    q.push_back(gi[p]);
                }
        }
        const int32_t ecc = level[q.back()];
        int32_t best = q.back();
        for (const int32_t v : q)
            if (level[v] == ecc && (deg[v] < deg[best] || (deg[v] == deg[best] && v < best))) best = v;
        *far = best;
        for (const int32_t v : q) level[v] = -1;
        return std::make_pair(ecc, std::move(q));
    };
    perm.clear();
    perm.reserve(n);
    std::vector<int32_t> nb;
    for (int64_t s0 = 0; s0 < n; ++s0) {
        if (done[s0]) continue;
        int32_t far = 0;
        const std::vector<int32_t> members = bfs((int32_t)s0, &far).second;
        int32_t r = members[0];
        for (const int32_t v : members)
            if (deg[v] < deg[r] || (deg[v] == deg[r] && v < r)) r = v;
        int32_t ecc = bfs(r, &far).first;
        for (;;) {
            int32_t far2 = 0;
            const int32_t e2 = bfs(far, &far2).first;
            if (e2 <= ecc) break;
            r = far;
            ecc = e2;
            far = far2;
        }
        const size_t head0 = perm.size();
        perm.push_back(r);
        done[r] = 1;
        for (size_t h = head0; h < perm.size(); ++h) {
            const int32_t v = perm[h];
            nb.clear();
            for (int64_t p = gp[v]; p < gp[v + 1]; ++p)
                if (!done[gi[p]]) {
                    done[gi[p]] = 1;
                    nb.push_back(gi[p]);
                }
            std::sort(nb.begin(), nb.end(),
                      [&](int32_t x, int32_t y) { return deg[x] < deg[y] || (deg[x] == deg[y] && x < y); });
            perm.insert(perm.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(perm.begin(), perm.end());
}

// ---------------------------------------------------------------------------------------
// Exact minimum degree: n times, take the live vertex whose current elimination-graph
// degree is smallest (ties: smallest index), make its live neighbours pairwise adjacent and
// remove it.  Priority: an ordered set of (degree, vertex); adjacency kept sorted.
// ---------------------------------------------------------------------------------------
void minimum_degree(int64_t n, const int64_t *rp, const int32_t *ci, std::vector<int32_t> &q) {
    std::vector<std::vector<int32_t>> nbr(n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] != i) {
                nbr[i].push_back(ci[p]);
                nbr[ci[p]].push_back((int32_t)i);
            }
    std::set<std::pair<int64_t, int32_t>> queue;
    for (int64_t v = 0; v < n; ++v) {
        auto &a = nbr[v];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        queue.emplace((int64_t)a.size(), (int32_t)v);
    }
    q.clear();
    q.reserve(n);
    std::vector<int32_t> scratch;
    while (!queue.empty()) {
        const int32_t v = queue.begin()->second;
        queue.erase(queue.begin());
        q.push_back(v);
        const std::vector<int32_t> clique = std::move(nbr[v]);
        nbr[v].clear();
        for (const int32_t u : clique) {
            auto &a = nbr[u];
            queue.erase({(int64_t)a.size(), u});
            scratch.clear();
            std::set_union(a.begin(), a.end(), clique.begin(), clique.end(), std::back_inserter(scratch));
            a.clear();
            for (const int32_t w : scratch)
                if (w != u && w != v) a.push_back(w);
            queue.emplace((int64_t)a.size(), u);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Left-looking LU of A(:,Q) with threshold partial pivoting.  For step j (column c = q[j]):
//  - x = A(:,c) by original row;
//  - structural closure from the rows of A(:,c): a row already pivoted at step k pulls in
//    every row of L(:,k); reached steps form U(:,j) above the diagonal, reached unpivoted
//    rows are the pivot candidates (all kept, zero or not);
//  - reached steps in ascending order: u = x[prow[k]], then x[i] = x[i] - L(i,k)*u;
//  - pivot: the diagonal row c if it is a candidate with |x_c| >= tau * max|x|, else the
//    candidate of largest |x| (ties: smallest row); max|x| == 0 is a singular column;
//  - U(j,j) = x[pivot]; L(i,j) = x[i] / U(j,j) for the other candidates.
// ---------------------------------------------------------------------------------------
int pivoted_lu(int64_t n, const int64_t *rp, const int32_t *ci, const double *val, double tau,
               Analysis &a, std::string *msg) {
    // column access to A
    std::vector<int64_t> cp(n + 1, 0);
    const int64_t nnz = rp[n];
    for (int64_t p = 0; p < nnz; ++p) ++cp[ci[p] + 1];
    for (int64_t c = 0; c < n; ++c) cp[c + 1] += cp[c];
    std::vector<int32_t> crow(nnz);
    std::vector<double> cval(nnz);
    {
        std::vector<int64_t> fillp(cp.begin(), cp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int64_t dst = fillp[ci[p]]++;
                crow[dst] = (int32_t)i;
                cval[dst] = val[p];
            }
    }
    a.prow.assign(n, -1);
    a.pinv.assign(n, -1);
    a.lp.assign(n + 1, 0);
    a.up.assign(n + 1, 0);
    a.li.clear();
    a.lx.clear();
    a.ui.clear();
    a.ux.clear();
    std::vector<double> x(n, 0.0);
    std::vector<int64_t> visited(n, -1);
    std::vector<int32_t> work, steps, cands;
    work.reserve(1024);
    int64_t offdiag = 0;
    for (int64_t j = 0; j < n; ++j) {
        const int32_t c = a.q[j];
        work.clear();
        steps.clear();
        cands.clear();
        for (int64_t p = cp[c]; p < cp[c + 1]; ++p) {
            x[crow[p]] = cval[p];
            visited[crow[p]] = j;
            work.push_back(crow[p]);
        }
        while (!work.empty()) {
            const int32_t r = work.back();
            work.pop_back();
            const int32_t k = a.pinv[r];
            if (k < 0) {
                cands.push_back(r);
                continue;
            }
            steps.push_back(k);
            for (int64_t p = a.lp[k]; p < a.lp[k + 1]; ++p) {
                const int32_t i = a.li[p];
                if (visited[i] != j) {
                    visited[i] = j;
                    work.push_back(i);
                }
            }
        }
        std::sort(steps.begin(), steps.end());
        for (int32_t k : steps) {
            const double u = x[a.prow[k]];
            a.ui.push_back(k);
            a.ux.push_back(u);
            for (int64_t p = a.lp[k]; p < a.lp[k + 1]; ++p) {
                const double t = a.lx[p] * u;
                x[a.li[p]] = x[a.li[p]] - t;
            }
        }
        std::sort(cands.begin(), cands.end());
        int32_t piv = -1;
        double amax = 0.0;
        for (int32_t r : cands) {
            const double m = std::fabs(x[r]);
            if (m > amax) {
                amax = m;
                piv = r;
            }
        }
        if (cands.empty() || !(amax > 0.0)) {
            *msg = "structurally or numerically singular at pivot step " + std::to_string(j) +
                   " (column " + std::to_string(c) + ")";
            return AN_ESINGULAR;
        }
        if (visited[c] == j && a.pinv[c] < 0 && std::fabs(x[c]) >= tau * amax) piv = c;
        if (piv != c) ++offdiag;
        const double d = x[piv];
        a.ui.push_back((int32_t)j);
        a.ux.push_back(d);
        a.up[j + 1] = (int64_t)a.ui.size();
        a.prow[j] = piv;
        a.pinv[piv] = (int32_t)j;
        for (int32_t r : cands) {
            if (r == piv) continue;
            a.li.push_back(r);
            a.lx.push_back(x[r] / d);
        }
        a.lp[j + 1] = (int64_t)a.li.size();
        for (int32_t r : cands) x[r] = 0.0;
        for (int32_t k : steps) x[a.prow[k]] = 0.0;
    }
    a.offdiag_pivots = offdiag;
    return AN_OK;
}

// Combined step-space factor F, the update positions, and the GPU schedules.
// Triangular-solve schedule.
//
// The rows form a DAG (row i waits for every row it references).  Level = longest path from
// a row without references.  Consecutive levels are grouped into *windows*; inside a window
// the rows split into weakly connected components (edges between rows of the window), which
// depend on each other only through earlier windows.  A component is solved by one block,
// level by level with a barrier in between, from LDS, so a chain of dependencies inside a
// window costs barriers, not cross-block waits.  A window grows one level at a time while
// every component still fits a staged tile (rows, LDS bytes for its entries and externals,
// each level covered by one pass of the block with at most `kSerial` entries per lane); a
// single level always forms a window (its rows are independent).  Components of a window
// are packed in order into tiles (next fit); a tile's rows at one level form a segment.  A
// row too long to stage on its own becomes an unstaged tile.
//
// Tiles are numbered window by window, so every reference of a tile is to a row of an
// earlier tile or of the same tile at an earlier segment.
bool tri_schedule(const AnalysisOptions &opt, int64_t n, const std::vector<int64_t> &rp,
                  const std::vector<int32_t> &ci, bool lower, int64_t dense_reserve, TriSchedule &sc,
                  std::string *msg) {
    constexpr int64_t kSerial = 16;  // entries per lane allowed when rows share a pass
    const int threads = opt.tile_threads;
    std::vector<int32_t> level(n, 0);
    if (lower) {
        for (int64_t i = 0; i < n; ++i) {
            int32_t l = 0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) l = std::max(l, level[ci[p]] + 1);
            level[i] = l;
        }
    } else {
        for (int64_t i = n - 1; i >= 0; --i) {
            int32_t l = 0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) l = std::max(l, level[ci[p]] + 1);
            level[i] = l;
        }
    }
    const int32_t nlev = n ? 1 + *std::max_element(level.begin(), level.end()) : 0;
    sc.levels = nlev;
    // rows by level; within a level in the direction of the sweep
    std::vector<int32_t> by_level(n);
    std::vector<int32_t> lev_ptr(nlev + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++lev_ptr[level[i] + 1];
    for (int32_t l = 0; l < nlev; ++l) lev_ptr[l + 1] += lev_ptr[l];
    {
        std::vector<int32_t> fill(lev_ptr.begin(), lev_ptr.end() - 1);
        for (int64_t s = 0; s < n; ++s) {
            const int32_t i = (int32_t)(lower ? s : n - 1 - s);
            by_level[fill[level[i]]++] = i;
        }
    }
    auto len = [&](int32_t i) { return rp[i + 1] - rp[i]; };
    auto lanes_needed = [&](int64_t m) {  // fewest lanes (power of two) with <= kSerial entries each
        int64_t g = 1;
        while (g < 64 && g * kSerial < m) g <<= 1;
        return g;
    };
    auto fits = [&](int64_t count, int64_t maxlen) { return count * lanes_needed(maxlen) <= threads; };

    // Components of a window, with per-level statistics, by union-find over the window's rows.
    struct LevStat {
        int32_t level, count;
        int64_t maxlen;
    };
    struct Size {
        int64_t rows = 0, ent = 0, ext = 0;  // ext: references to earlier windows (upper bound)
    };
    // Tiles of a window that starts at a narrow level (the top of the DAG, where runs of small
    // levels become dense segments) are formed within a smaller budget, so that dense blocks
    // fit in what remains; wide windows use the whole budget (fewer, larger tiles: at 2M
    // unknowns the reserve in every window made the L sweep 30 % slower).
    auto budget_at = [&](int32_t l) {
        return lev_ptr[l + 1] - lev_ptr[l] <= kDenseWindowRows ? opt.tile_lds - dense_reserve : opt.tile_lds;
    };
    int64_t stage_budget = budget_at(0);
    auto stageable = [&](const Size &z) {
        return z.rows <= opt.tile_rows && tile_lds_bytes(z.rows, z.ext, z.ent) <= stage_budget;
    };
    std::vector<int32_t> parent(n, -1);
    std::vector<Size> size(n);
    std::vector<std::vector<LevStat>> stat(n);
    auto find = [&](int32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    };
    // merges the components of x and y (the smaller level list into the larger, in place);
    // returns false when the result no longer fits a tile
    auto unite = [&](int32_t x, int32_t y) {
        x = find(x);
        y = find(y);
        if (x == y) return true;
        if (stat[x].size() < stat[y].size()) std::swap(x, y);
        std::vector<LevStat> &big = stat[x];
        bool ok = true;
        for (const LevStat &e : stat[y]) {
            auto it = std::lower_bound(big.begin(), big.end(), e.level,
                                       [](const LevStat &a, int32_t l) { return a.level < l; });
            if (it != big.end() && it->level == e.level) {
                it->count += e.count;
                it->maxlen = std::max(it->maxlen, e.maxlen);
            } else {
                it = big.insert(it, e);
            }
            ok = ok && fits(it->count, it->maxlen);
        }
        parent[y] = x;
        size[x].rows += size[y].rows;
        size[x].ent += size[y].ent;
        size[x].ext += size[y].ext;
        std::vector<LevStat>().swap(stat[y]);
        return ok && stageable(size[x]);
    };
    auto add_level = [&](int32_t l, int32_t w0) {
        bool ok = true;
        for (int32_t r = lev_ptr[l]; r < lev_ptr[l + 1]; ++r) {
            const int32_t i = by_level[r];
            parent[i] = i;
            Size z;
            z.rows = 1;
            z.ent = len(i);
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) z.ext += level[ci[p]] < w0;
            size[i] = z;
            stat[i].assign(1, LevStat{l, 1, len(i)});
        }
        for (int32_t r = lev_ptr[l]; r < lev_ptr[l + 1]; ++r) {
            const int32_t i = by_level[r];
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (level[ci[p]] >= w0 && !unite(i, ci[p])) ok = false;
        }
        return ok;
    };
    auto clear_window = [&](int32_t w0, int32_t w1) {
        for (int32_t r = lev_ptr[w0]; r < lev_ptr[w1 + 1]; ++r) {
            const int32_t i = by_level[r];
            parent[i] = -1;
            std::vector<LevStat>().swap(stat[i]);
        }
    };

    sc.rows.clear();
    sc.rows.reserve(n);
    sc.tile_seg.assign(1, 0);
    sc.seg_row.assign(1, 0);
    sc.seg_lg.clear();
    sc.tile_lds.clear();
    sc.seg_dofs.clear();
    std::vector<int64_t> tile_dvals;  // dense-block values of each tile
    sc.windows = 0;
    std::vector<int32_t> tcount, comp_of_root(n, -1);
    std::vector<int64_t> tmax;
    // packs the components of window [w0, w1] into tiles
    auto emit_window = [&](int32_t w0, int32_t w1) {
        ++sc.windows;
        const int32_t nl = w1 - w0 + 1;
        // components in order of their first row (level-major order)
        std::vector<int32_t> roots;
        for (int32_t r = lev_ptr[w0]; r < lev_ptr[w1 + 1]; ++r) {
            const int32_t x = find(by_level[r]);
            if (comp_of_root[x] < 0) {
                comp_of_root[x] = (int32_t)roots.size();
                roots.push_back(x);
            }
        }
        // rows of each component (level-major, sweep order inside a level)
        std::vector<std::vector<int32_t>> crows(roots.size());
        for (int32_t r = lev_ptr[w0]; r < lev_ptr[w1 + 1]; ++r) {
            const int32_t i = by_level[r];
            crows[comp_of_root[find(i)]].push_back(i);
        }
        tcount.assign(nl, 0);
        tmax.assign(nl, 0);
        Size tsize;
        std::vector<int32_t> members;
        auto lane_log = [&](int64_t cnt, int64_t maxlen, int64_t pass) {
            int lg = 0;  // about four entries per lane, at most 64 lanes, one pass
            while (lg < 6 && ((int64_t)1 << lg) * 4 < maxlen) ++lg;
            while (lg > 0 && (cnt << lg) > pass) --lg;
            return lg;
        };
        auto close_tile = [&](bool staged) {
            if (members.empty()) return;
            // the tile's levels: rows in order, counts and longest rows
            std::vector<int32_t> lcnt;
            std::vector<int64_t> lmax;
            for (int32_t l = w0; l <= w1; ++l) {
                const int32_t cnt = tcount[l - w0];
                if (!cnt) continue;
                for (int32_t c : members)
                    for (int32_t i : crows[c])
                        if (level[i] == l) sc.rows.push_back(i);
                lcnt.push_back(cnt);
                lmax.push_back(tmax[l - w0]);
                tcount[l - w0] = 0;
                tmax[l - w0] = 0;
            }
            // consecutive small levels are fused into dense segments while the LDS left over
            // by the tile's entries holds their blocks, in windows that start at a narrow level
            // only (fused blocks in the tiles of wide windows made the 2M L sweep 4 % slower)
            int64_t room = staged && dense_reserve > 0 && stage_budget < opt.tile_lds
                               ? opt.tile_lds - tile_lds_bytes(tsize.rows, tsize.ext, tsize.ent)
                               : 0;
            int64_t dvals = 0;
            int32_t row = sc.seg_row.back();
            for (size_t k = 0; k < lcnt.size();) {
                size_t k1 = k + 1;
                int64_t m = lcnt[k], mx = lmax[k];
                while (k1 < lcnt.size() && m + lcnt[k1] <= kDenseRows &&
                       8 * dense_block_values(m + lcnt[k1]) <= room) {
                    m += lcnt[k1];
                    mx = std::max(mx, lmax[k1]);
                    ++k1;
                }
                // worth it only when the levels it replaces cost more than its sweep: about
                // one segment per level against 1.5 segments plus m / 32 for the sweep
                if (k1 - k >= 2 && 32 * (int64_t)(k1 - k) < 48 + m) {
                    k1 = k + 1;
                    m = lcnt[k];
                    mx = lmax[k];
                }
                row += (int32_t)m;
                sc.seg_row.push_back(row);
                if (k1 - k >= 2) {  // dense segment: phase A is a block pass over its rows
                    sc.seg_lg.push_back(lane_log(m, mx, threads) | kSegDense);
                    sc.seg_dofs.push_back((int32_t)dvals);
                    dvals += dense_block_values(m);
                    room -= 8 * dense_block_values(m);
                } else {
                    // a wavefront pass when it covers the level with these lanes (no block
                    // barrier needed), else a block pass with fewer lanes per row if needed
                    const int lgw = lane_log(m, mx, 64 * 64);
                    const bool wave = (m << lgw) <= 64;
                    sc.seg_lg.push_back(lane_log(m, mx, threads) | (wave ? kSegWave : 0));
                    sc.seg_dofs.push_back(-1);
                }
                k = k1;
            }
            sc.tile_seg.push_back((int32_t)sc.seg_lg.size());
            sc.tile_lds.push_back(staged ? 1 : 0);
            tile_dvals.push_back(dvals);
            members.clear();
            tsize = Size();
        };
        for (size_t c = 0; c < roots.size(); ++c) {
            const std::vector<LevStat> &st = stat[roots[c]];
            const Size &z = size[roots[c]];
            if (!stageable(z)) {  // a single row too long to stage: a tile of its own
                close_tile(true);
                members.push_back((int32_t)c);
                for (const LevStat &e : st) {
                    tcount[e.level - w0] += e.count;
                    tmax[e.level - w0] = std::max(tmax[e.level - w0], e.maxlen);
                }
                close_tile(false);
                continue;
            }
            Size sum = tsize;
            sum.rows += z.rows;
            sum.ent += z.ent;
            sum.ext += z.ext;
            bool ok = stageable(sum);
            for (size_t e = 0; ok && e < st.size(); ++e) {
                const int32_t k = st[e].level - w0;
                ok = fits(tcount[k] + st[e].count, std::max(tmax[k], st[e].maxlen));
            }
            if (!ok) {
                close_tile(true);
                sum = z;
            }
            for (const LevStat &e : st) {
                tcount[e.level - w0] += e.count;
                tmax[e.level - w0] = std::max(tmax[e.level - w0], e.maxlen);
            }
            tsize = sum;
            members.push_back((int32_t)c);
        }
        close_tile(true);
        for (int32_t x : roots) comp_of_root[x] = -1;
    };

    int32_t w0 = 0;
    for (int32_t l = 0; l < nlev; ++l) {
        if (add_level(l, w0) || l == w0) continue;
        // level l does not fit the window: rebuild the window without it, emit it, and start
        // a new window at l
        clear_window(w0, l);
        for (int32_t k = w0; k < l; ++k) add_level(k, w0);
        emit_window(w0, l - 1);
        clear_window(w0, l - 1);
        w0 = l;
        stage_budget = budget_at(l);
        add_level(l, w0);
    }
    if (nlev) emit_window(w0, nlev - 1);
    if ((int64_t)sc.rows.size() != n) {
        *msg = "internal: triangular schedule lost rows";
        return false;
    }
    // packed entries, externals and references
    std::vector<int32_t> pos(n), tile_of(n), seg_of(n);
    for (int64_t r = 0; r < n; ++r) pos[sc.rows[r]] = (int32_t)r;
    for (int64_t t = 0; t < sc.tiles(); ++t)
        for (int32_t g = sc.tile_seg[t]; g < sc.tile_seg[t + 1]; ++g)
            for (int32_t r = sc.seg_row[g]; r < sc.seg_row[g + 1]; ++r) {
                tile_of[r] = (int32_t)t;
                seg_of[r] = g;
            }
    // dense segments: local index of each position, and whether a reference stays inside
    std::vector<int32_t> dloc(n, -1);
    for (int64_t g = 0; g < sc.segments(); ++g)
        if (sc.seg_lg[g] & kSegDense)
            for (int32_t r = sc.seg_row[g]; r < sc.seg_row[g + 1]; ++r) dloc[r] = r - sc.seg_row[g];
    auto inside = [&](int32_t r, int32_t pk) { return dloc[r] >= 0 && seg_of[pk] == seg_of[r]; };
    sc.row_ent.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        const int32_t i = sc.rows[r];
        int64_t cnt = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) cnt += !inside((int32_t)r, pos[ci[p]]);
        sc.row_ent[r + 1] = sc.row_ent[r] + cnt;
    }
    sc.packed = sc.row_ent[n];
    sc.tile_dense.assign(1, sc.packed);
    for (int64_t t = 0; t < sc.tiles(); ++t) sc.tile_dense.push_back(sc.tile_dense.back() + tile_dvals[t]);
    sc.ent_ref.assign(sc.packed, 0);
    sc.csr2ent.assign(ci.size(), 0);
    sc.tile_ext.assign(1, 0);
    sc.ext_src.clear();
    std::vector<int32_t> ext_slot(n, -1);
    for (int64_t t = 0; t < sc.tiles(); ++t) {
        const int32_t rb = sc.seg_row[sc.tile_seg[t]], re = sc.seg_row[sc.tile_seg[t + 1]];
        const size_t x0 = sc.ext_src.size();
        for (int32_t r = rb; r < re; ++r) {
            const int32_t i = sc.rows[r];
            int64_t e = sc.row_ent[r];
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t k = ci[p];
                const int32_t pk = pos[k];
                if (tile_of[pk] > t || (seg_of[pk] >= seg_of[r] && !(inside(r, pk) && pk < r))) {
                    *msg = "internal: triangular schedule order";
                    return false;
                }
                if (inside(r, pk)) {  // column-major strictly lower dense block, local (r, c)
                    const int64_t g = seg_of[r];
                    const int64_t m = sc.seg_row[g + 1] - sc.seg_row[g];
                    const int64_t lr = dloc[r], lc = dloc[pk];
                    sc.csr2ent[p] = sc.tile_dense[t] + sc.seg_dofs[g] + lc * m - lc * (lc + 1) / 2 + (lr - lc - 1);
                    continue;
                }
                sc.csr2ent[p] = e;
                if (!sc.tile_lds[t]) {
                    sc.ent_ref[e] = k;
                } else if (tile_of[pk] == t) {
                    sc.ent_ref[e] = pk - rb;
                } else {
                    if (ext_slot[k] < 0) {
                        ext_slot[k] = (int32_t)(sc.ext_src.size() - x0);
                        sc.ext_src.push_back(k);
                    }
                    sc.ent_ref[e] = (re - rb) + ext_slot[k];
                }
                ++e;
            }
        }
        for (size_t k = x0; k < sc.ext_src.size(); ++k) ext_slot[sc.ext_src[k]] = -1;
        sc.tile_ext.push_back((int32_t)sc.ext_src.size());
        if (sc.tile_lds[t] &&
            tile_lds_bytes(re - rb, (int64_t)(sc.ext_src.size() - x0), sc.row_ent[re] - sc.row_ent[rb],
                           tile_dvals[t]) > opt.tile_lds) {
            *msg = "internal: staged tile exceeds its LDS budget";
            return false;
        }
    }
    return true;
}

int build_layouts(const AnalysisOptions &opt, Analysis &a, std::string *msg) {
    const int64_t n = a.n;
    const int64_t lnz = a.nnz_l(), unz = a.nnz_u();
    const int64_t f = lnz + unz;
    if (f >= (int64_t)std::numeric_limits<int32_t>::max()) {
        *msg = "factor too large for 32-bit positions";
        return AN_ENOMEM;
    }
    // --- F columns: U part (steps ascending, without the diagonal), diagonal, L part
    // (steps ascending).  L(:,j) is stored by original row; sort its step indices.
    a.fp.assign(n + 1, 0);
    a.fi.resize(f);
    a.fx.resize(f);
    a.fdiag.resize(n);
    a.l2f.resize(lnz);
    a.u2f.resize(unz);
    std::vector<std::pair<int32_t, int64_t>> lpart;
    int64_t w = 0;
    for (int64_t j = 0; j < n; ++j) {
        a.fp[j] = w;
        for (int64_t p = a.up[j]; p < a.up[j + 1]; ++p) {
            a.fi[w] = a.ui[p];
            a.fx[w] = a.ux[p];
            a.u2f[p] = w;
            ++w;
        }
        a.fdiag[j] = (int32_t)(a.up[j + 1] - a.up[j] - 1);
        lpart.clear();
        for (int64_t p = a.lp[j]; p < a.lp[j + 1]; ++p) lpart.emplace_back(a.pinv[a.li[p]], p);
        std::sort(lpart.begin(), lpart.end());
        for (auto &e : lpart) {
            a.fi[w] = e.first;
            a.fx[w] = a.lx[e.second];
            a.l2f[e.second] = w;
            ++w;
        }
    }
    a.fp[n] = w;
    // --- ingest gather map: F entry of (step row r, step col j) takes K(prow[r], q[j])
    a.fsrc.assign(f, -1);
    {
        std::vector<int64_t> at(n, -1);  // step row -> F position within the current column
        std::vector<int32_t> qinv(n);
        for (int64_t j = 0; j < n; ++j) qinv[a.q[j]] = (int32_t)j;
        // process K by original column: transpose view
        std::vector<int64_t> cp(n + 1, 0);
        for (int64_t p = 0; p < a.nnz; ++p) ++cp[a.colidx[p] + 1];
        for (int64_t c = 0; c < n; ++c) cp[c + 1] += cp[c];
        std::vector<int64_t> src(a.nnz);
        std::vector<int32_t> srow(a.nnz);
        std::vector<int64_t> fillp(cp.begin(), cp.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
                const int64_t d = fillp[a.colidx[p]]++;
                src[d] = p;
                srow[d] = (int32_t)i;
            }
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) at[a.fi[t]] = t;
            const int32_t c = a.q[j];
            for (int64_t d = cp[c]; d < cp[c + 1]; ++d) {
                const int64_t t = at[a.pinv[srow[d]]];
                if (t < a.fp[j] || t >= a.fp[j + 1] || a.fi[t] != a.pinv[srow[d]]) {
                    *msg = "internal: entry of K outside the factor pattern";
                    return AN_EINVAL;
                }
                a.fsrc[t] = src[d];
            }
        }
    }
    // --- update positions and refactorization levels
    {
        int64_t total = 0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t t = a.fp[j]; t < a.fp[j] + a.fdiag[j]; ++t) {
                const int32_t k = a.fi[t];
                total += a.fp[k + 1] - (a.fp[k] + a.fdiag[k] + 1);
            }
        a.relptr.assign(n + 1, 0);
        a.relpos.resize(total);
        const bool flat = a.nnz_f() < ((int64_t)1 << 31);
        a.relsrc.assign(flat ? total : 0, 0);
        a.relslot.assign(flat ? total : 0, 0);
        std::vector<int32_t> where(n, -1);
        std::vector<int64_t> level(n, 0);
        int64_t r = 0;
        for (int64_t j = 0; j < n; ++j) {
            a.relptr[j] = r;
            for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) where[a.fi[t]] = (int32_t)(t - a.fp[j]);
            int64_t lev = 0;
            for (int64_t t = a.fp[j]; t < a.fp[j] + a.fdiag[j]; ++t) {
                const int32_t k = a.fi[t];
                lev = std::max(lev, level[k] + 1);
                for (int64_t s = a.fp[k] + a.fdiag[k] + 1; s < a.fp[k + 1]; ++s) {
                    const int32_t pos = where[a.fi[s]];
                    if (pos < 0 || a.fi[a.fp[j] + pos] != a.fi[s]) {
                        *msg = "internal: update outside the factor pattern";
                        return AN_EINVAL;
                    }
                    if (flat) {
                        a.relsrc[r] = (int32_t)s;
                        a.relslot[r] = (int32_t)(t - a.fp[j]);
                    }
                    a.relpos[r++] = pos;
                }
            }
            level[j] = lev;
            for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) where[a.fi[t]] = -1;
        }
        a.relptr[n] = r;
        // columns by (level, lane-sized first, index)
        // (lane-sized columns of a level by ascending update count, so that the 64 lanes of an
        // item have about the same work; columns of one level are independent, so their order
        // is free.  Ordering them by their position in the vector order, for locality, measured
        // no faster at 2M unknowns and slower at 60k.)
        auto lane_sized = [&](int32_t j) { return flat && a.fp[j + 1] - a.fp[j] <= kLaneLen; };
        a.col_order.resize(n);
        for (int64_t j = 0; j < n; ++j) a.col_order[j] = (int32_t)j;
        std::stable_sort(a.col_order.begin(), a.col_order.end(), [&](int32_t x, int32_t y) {
            if (level[x] != level[y]) return level[x] < level[y];
            const bool lx = lane_sized(x), ly = lane_sized(y);
            if (lx != ly) return lx;
            if (lx) return a.relptr[x + 1] - a.relptr[x] < a.relptr[y + 1] - a.relptr[y];
            return false;
        });
        a.col_level.resize(n);
        for (int64_t t = 0; t < n; ++t) a.col_level[t] = (int32_t)level[a.col_order[t]];
        a.levels_refactor = n ? 1 + *std::max_element(level.begin(), level.end()) : 0;
        std::vector<int64_t> width(a.levels_refactor + 1, 0);
        for (int64_t j = 0; j < n; ++j) ++width[level[j]];
        a.ref_item.clear();
        a.ref_item_lane.clear();
        for (int64_t p0 = 0; p0 < n;) {
            const int64_t l = level[a.col_order[p0]];
            const int64_t p1 = p0 + width[l];
            const bool wide = width[l] > opt.narrow_columns;
            int64_t pe = p0;
            while (wide && pe < p1 && lane_sized(a.col_order[pe])) ++pe;
            for (int64_t t = p0; t < pe; t += 64) {
                a.ref_item.push_back((int32_t)t);
                a.ref_item_lane.push_back(1);
            }
            const int64_t step = wide ? kLaneChunk : 1;
            for (int64_t t = pe; t < p1; t += step) {
                a.ref_item.push_back((int32_t)t);
                a.ref_item_lane.push_back(0);
            }
            p0 = p1;
        }
        a.ref_item.push_back((int32_t)n);
        // a wavefront runs a lane item's columns together, so none may wait for another: one
        // level, at most 64 columns of at most kLaneLen entries (checked, since a violation
        // would stall the refactorization until its spin limit)
        for (size_t t = 0; t + 1 < a.ref_item.size(); ++t) {
            const int64_t b = a.ref_item[t], e = a.ref_item[t + 1];
            bool ok = e > b;
            if (a.ref_item_lane[t]) {
                ok = ok && e - b <= 64;
                for (int64_t q = b; ok && q < e; ++q)
                    ok = a.col_level[q] == a.col_level[b] && lane_sized(a.col_order[q]);
            } else {
                ok = ok && e - b <= kLaneChunk && a.col_level[e - 1] == a.col_level[b];
            }
            if (!ok) {
                *msg = "internal: refactorization hand-out item " + std::to_string(t);
                return AN_EINVAL;
            }
        }
    }
    // --- solve layout: L strict CSR, U strict CSR, diagonal; map F -> T
    {
        a.lrp.assign(n + 1, 0);
        a.urp.assign(n + 1, 0);
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t t = a.fp[j]; t < a.fp[j] + a.fdiag[j]; ++t) ++a.urp[a.fi[t] + 1];
            for (int64_t t = a.fp[j] + a.fdiag[j] + 1; t < a.fp[j + 1]; ++t) ++a.lrp[a.fi[t] + 1];
        }
        for (int64_t i = 0; i < n; ++i) {
            a.lrp[i + 1] += a.lrp[i];
            a.urp[i + 1] += a.urp[i];
        }
        a.lci.resize(a.lrp[n]);
        a.uci.resize(a.urp[n]);
        a.f2t.resize(f);
        std::vector<int64_t> lnext(a.lrp.begin(), a.lrp.end() - 1), unext(a.urp.begin(), a.urp.end() - 1);
        const int64_t ubase = a.lrp[n], dbase = a.lrp[n] + a.urp[n];
        for (int64_t j = 0; j < n; ++j) {  // columns ascending -> column indices ascending per row
            for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) {
                const int32_t r = a.fi[t];
                if (r < j) {
                    const int64_t d = unext[r]++;
                    a.uci[d] = (int32_t)j;
                    a.f2t[t] = (int32_t)(ubase + d);
                } else if (r == j) {
                    a.f2t[t] = (int32_t)(dbase + j);
                } else {
                    const int64_t d = lnext[r]++;
                    a.lci[d] = (int32_t)j;
                    a.f2t[t] = (int32_t)d;
                }
            }
        }
    }
    // --- triangular-solve schedules; T then holds each triangle's entries packed in solve
    // order (L, then strict U), followed by the diagonal of U in step order
    if (!tri_schedule(opt, n, a.lrp, a.lci, true, opt.dense_reserve_l, a.lsched, msg) ||
        !tri_schedule(opt, n, a.urp, a.uci, false, opt.dense_reserve_u, a.usched, msg))
        return AN_EINVAL;
    {
        const int64_t ubase = a.lrp[n], dbase = a.lrp[n] + a.urp[n];
        const int64_t tu = a.lsched.values(), td = tu + a.usched.values();
        for (int64_t t = 0; t < f; ++t) {
            const int64_t d = a.f2t[t];
            if (d < ubase) a.f2t[t] = (int32_t)a.lsched.csr2ent[d];
            else if (d < dbase) a.f2t[t] = (int32_t)(tu + a.usched.csr2ent[d - ubase]);
            else a.f2t[t] = (int32_t)(td + (d - dbase));
        }
        a.t_size = td + n;
    }
    return AN_OK;
}

// The Krylov side's copy of K in the vector order vperm (reverse Cuthill-McKee): row k is
// original row vperm[k] with its entries in their original order and columns renumbered, the
// source position of every entry, the factor entries' sources in that copy, and the pivot
// permutations composed with it.
void build_vector_order(Analysis &a) {
    const int64_t n = a.n, nnz = a.nnz;
    a.krp.assign(n + 1, 0);
    a.kci.resize(nnz);
    a.ksrc.resize(nnz);
    std::vector<int64_t> epos(nnz);
    int64_t w = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int32_t i = a.vperm[k];
        a.krp[k] = w;
        for (int64_t p = a.rowptr[i]; p < a.rowptr[i + 1]; ++p) {
            a.kci[w] = a.vpinv[a.colidx[p]];
            a.ksrc[w] = p;
            epos[p] = w++;
        }
    }
    a.krp[n] = w;
    a.fsrc_k.resize(a.fsrc.size());
    for (size_t t = 0; t < a.fsrc.size(); ++t) a.fsrc_k[t] = a.fsrc[t] >= 0 ? epos[a.fsrc[t]] : -1;
    a.prow_k.resize(n);
    a.q_k.resize(n);
    for (int64_t k = 0; k < n; ++k) {
        a.prow_k[k] = a.vpinv[a.prow[k]];
        a.q_k[k] = a.vpinv[a.q[k]];
    }
}

// The device layout of the flat refactorization (see Analysis::phys): F positions and update
// lists renumbered in col_order.
void build_phys_layout(Analysis &a) {
    const int64_t n = a.n, f = a.nnz_f();
    std::vector<int64_t> phys(f);
    a.pc.assign(n + 1, 0);
    a.pu.assign(n + 1, 0);
    a.pnu.assign(n, 0);
    int64_t w = 0, u = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t j = a.col_order[p];
        a.pc[p] = w;
        a.pu[p] = u;
        a.pnu[p] = a.fdiag[j];
        for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) phys[t] = w++;
        u += a.relptr[j + 1] - a.relptr[j];
    }
    a.pc[n] = w;
    a.pu[n] = u;
    std::vector<int32_t> rpos(a.relpos.size()), rsrc(a.relsrc.size()), rslot(a.relslot.size());
    for (int64_t p = 0; p < n; ++p) {
        const int32_t j = a.col_order[p];
        for (int64_t k = a.relptr[j], d = a.pu[p]; k < a.relptr[j + 1]; ++k, ++d) {
            rpos[d] = a.relpos[k];
            rsrc[d] = (int32_t)phys[a.relsrc[k]];
            rslot[d] = a.relslot[k];
        }
    }
    a.relpos.swap(rpos);
    a.relsrc.swap(rsrc);
    a.relslot.swap(rslot);
    std::vector<int32_t> f2t(f);
    std::vector<int64_t> fsrc(f);
    for (int64_t t = 0; t < f; ++t) {
        f2t[phys[t]] = a.f2t[t];
        fsrc[phys[t]] = a.fsrc_k[t];
    }
    a.f2t.swap(f2t);
    a.fsrc_k.swap(fsrc);
    for (auto &t : a.l2f) t = phys[t];
    for (auto &t : a.u2f) t = phys[t];
    a.phys = true;
}

}  // namespace

void vector_order(int64_t n, const int64_t *rowptr, const int32_t *colidx, std::vector<int32_t> &perm) {
    rcm_order(n, rowptr, colidx, perm);
}

int nested_dissection(int64_t n, const int64_t *rowptr, const int32_t *colidx, int64_t leaf,
                      std::vector<int32_t> &q) {
    Dissector d(n, rowptr, colidx, leaf < 1 ? 1 : leaf);
    d.run(q);
    return (int64_t)q.size() == n ? AN_OK : AN_EINVAL;
}

int analyze(const AnalysisOptions &opt, int64_t n, const int64_t *rowptr, const int32_t *colidx,
            const double *values, Analysis &a, std::string *msg) {
    const auto t0 = std::chrono::steady_clock::now();
    try {
        if (!rowptr || !colidx || !values) {
            *msg = "null input pointer";
            return AN_EINVAL;
        }
        if (!csr_valid(n, rowptr, colidx, msg)) return AN_EINVAL;
        for (int64_t p = 0; p < rowptr[n]; ++p)
            if (!std::isfinite(values[p])) {
                *msg = "non-finite value at position " + std::to_string(p);
                return AN_EINVAL;
            }
        a = Analysis();
        a.n = n;
        a.nnz = rowptr[n];
        a.rowptr.assign(rowptr, rowptr + n + 1);
        a.colidx.assign(colidx, colidx + a.nnz);
        int rc = AN_OK;
        if (opt.fixed_order) a.q.assign(opt.fixed_order, opt.fixed_order + n);
        else if (opt.ordering == ORDER_ND) rc = nested_dissection(n, rowptr, colidx, opt.nd_leaf, a.q);
        else minimum_degree(n, rowptr, colidx, a.q);
        if (rc != AN_OK || (int64_t)a.q.size() != n) {
            *msg = "ordering failed";
            return AN_EINVAL;
        }
        rc = pivoted_lu(n, rowptr, colidx, values, opt.pivot_tau, a, msg);
        if (rc != AN_OK) return rc;
        rcm_order(n, rowptr, colidx, a.vperm);
        a.vpinv.assign(n, 0);
        for (int64_t k = 0; k < n; ++k) a.vpinv[a.vperm[k]] = (int32_t)k;
        rc = build_layouts(opt, a, msg);
        if (rc != AN_OK) return rc;
        build_vector_order(a);
        if (!a.relsrc.empty()) build_phys_layout(a);
    } catch (const std::bad_alloc &) {
        *msg = "out of host memory";
        return AN_ENOMEM;
    }
    a.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return AN_OK;
}

}  // namespace kkt
