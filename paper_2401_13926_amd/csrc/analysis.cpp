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
                    a.relpos[r++] = pos;
                }
            }
            level[j] = lev;
            for (int64_t t = a.fp[j]; t < a.fp[j + 1]; ++t) where[a.fi[t]] = -1;
        }
        a.relptr[n] = r;
        a.col_order.resize(n);
        for (int64_t j = 0; j < n; ++j) a.col_order[j] = (int32_t)j;
        std::stable_sort(a.col_order.begin(), a.col_order.end(),
                         [&](int32_t x, int32_t y) { return level[x] < level[y]; });
        a.levels_refactor = n ? 1 + *std::max_element(level.begin(), level.end()) : 0;
        std::vector<int64_t> width(a.levels_refactor + 1, 0);
        for (int64_t j = 0; j < n; ++j) ++width[level[j]];
        a.refactor_split = n;
        int64_t pos = 0;
        for (int64_t l = 0; l < a.levels_refactor; ++l) {
            if (width[l] <= opt.narrow_columns) {
                a.refactor_split = pos;
                break;
            }
            pos += width[l];
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
    // --- triangular-solve schedules
    auto schedule = [&](bool lower, TriSchedule &sc) {
        const std::vector<int64_t> &rp = lower ? a.lrp : a.urp;
        const std::vector<int32_t> &ci = lower ? a.lci : a.uci;
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
        sc.rows.resize(n);
        for (int64_t i = 0; i < n; ++i) sc.rows[i] = (int32_t)(lower ? i : n - 1 - i);
        std::stable_sort(sc.rows.begin(), sc.rows.end(), [&](int32_t x, int32_t y) { return level[x] < level[y]; });
        sc.lev_ptr.assign(nlev + 1, 0);
        for (int64_t i = 0; i < n; ++i) ++sc.lev_ptr[level[i] + 1];
        for (int32_t l = 0; l < nlev; ++l) sc.lev_ptr[l + 1] += sc.lev_ptr[l];
        sc.lev_lg.assign(nlev, 0);
        for (int32_t l = 0; l < nlev; ++l) {
            int64_t mx = 0;
            for (int32_t r = sc.lev_ptr[l]; r < sc.lev_ptr[l + 1]; ++r)
                mx = std::max(mx, rp[sc.rows[r] + 1] - rp[sc.rows[r]]);
            int lg = 0;  // lanes such that each lane handles about four entries, at most 64
            while (lg < 6 && ((int64_t)1 << lg) * 4 < mx) ++lg;
            sc.lev_lg[l] = (int8_t)lg;
        }
        // tiles
        sc.tile_row.assign(1, 0);
        sc.tile_lev.clear();
        int32_t open_rows = 0;  // rows in the current multi-level tile
        auto close = [&](int32_t end) {
            if (end > sc.tile_row.back()) sc.tile_row.push_back(end);
        };
        for (int32_t l = 0; l < nlev; ++l) {
            const int32_t r0 = sc.lev_ptr[l], r1 = sc.lev_ptr[l + 1];
            const int32_t cnt = r1 - r0;
            // a level joins a multi-level tile only when one pass of the block covers it
            // (each lane group then owns at most one row of the level)
            if (cnt > opt.narrow_rows || cnt > (opt.tile_threads >> sc.lev_lg[l])) {
                close(r0);
                open_rows = 0;
                const int32_t chunk = std::max(1, opt.tile_threads >> sc.lev_lg[l]);
                for (int32_t s0 = r0; s0 < r1; s0 += chunk) {
                    sc.tile_lev.push_back(l);
                    close(std::min(s0 + chunk, r1));
                }
                continue;
            }
            if (open_rows > 0 && open_rows + cnt > opt.tile_rows) {
                close(r0);
                open_rows = 0;
            }
            if (open_rows == 0) sc.tile_lev.push_back(l);
            open_rows += cnt;
        }
        close((int32_t)n);
        if ((int64_t)sc.tile_lev.size() != sc.tiles()) {
            *msg = "internal: tile bookkeeping";
            return false;
        }
        // encoded references
        std::vector<int32_t> pos(n), tile_of(n);
        for (int64_t r = 0; r < n; ++r) pos[sc.rows[r]] = (int32_t)r;
        for (int64_t t = 0; t < sc.tiles(); ++t)
            for (int32_t r = sc.tile_row[t]; r < sc.tile_row[t + 1]; ++r) tile_of[r] = (int32_t)t;
        sc.ref.resize(ci.size());
        for (int64_t i = 0; i < n; ++i) {
            const int32_t ti = tile_of[pos[i]];
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t k = ci[p];
                const int32_t pk = pos[k];
                sc.ref[p] = tile_of[pk] == ti ? -(pk - sc.tile_row[ti] + 1) : k;
            }
        }
        return true;
    };
    if (!schedule(true, a.lsched) || !schedule(false, a.usched)) return AN_EINVAL;
    return AN_OK;
}

}  // namespace

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
        if (opt.ordering == ORDER_ND) rc = nested_dissection(n, rowptr, colidx, opt.nd_leaf, a.q);
        else minimum_degree(n, rowptr, colidx, a.q);
        if (rc != AN_OK || (int64_t)a.q.size() != n) {
            *msg = "ordering failed";
            return AN_EINVAL;
        }
        rc = pivoted_lu(n, rowptr, colidx, values, opt.pivot_tau, a, msg);
        if (rc != AN_OK) return rc;
        rc = build_layouts(opt, a, msg);
        if (rc != AN_OK) return rc;
    } catch (const std::bad_alloc &) {
        *msg = "out of host memory";
        return AN_ENOMEM;
    }
    a.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return AN_OK;
}

}  // namespace kkt
