// HyKKT (Section 5, eq. (kktlineargamma)): KKT systems [[H + D, J^T], [J, 0]] with a zero (2,2)
// block solved through H_gamma = H + D + gamma J^T J (symmetric positive definite) and
// conjugate gradients on the Schur complement S = J H_gamma^-1 J^T, applied as products:
//
//   rhat = r_x + gamma J^T r_l,   S dl = J H_gamma^-1 rhat - r_l,   dx = H_gamma^-1 (rhat - J^T dl).
//
// The pattern of H_gamma (that of H + D joined with the structural pattern of J^T J) and the
// map from K's values to its entries are built once on the host ("SpGEMM" with a fixed
// pattern); per system one kernel forms the entries, and the LU refactorization of this
// library (diagonal pivots on the SPD matrix, i.e. Cholesky up to the diagonal scaling)
// refactors H_gamma with the analysis of the first system.  H_gamma^-1 is applied with the
// library's staged triangular solves (kkt_direct_solve).  Every reduction of the CG runs in
// a fixed order (per-block partial sums reduced by the next kernel), so solves are bitwise
// repeatable.  The host reads the CG's stop flag once per group of iterations; iterations
// enqueued past the stop do nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/kkt.h"

namespace {

constexpr int kBlock = 256;
constexpr int kGridMax = 1024;
constexpr int kCgGroup = 8;  // CG iterations enqueued between two reads of the stop flag

// Scalars of one solve (device memory).  Partial sums: block b writes part[b * 4 + t].
struct CgControl {
    double rr;      // r.r of the current iterate
    double rr_new;  // r.r after this iteration's update (moved to rr by k_hy_cg_finish)
    double rr0;     // r.r at the start
    double tol2;    // (cg_tol^2) rr0: stop when rr <= tol2
    int stop;       // CG finished (converged, iteration cap, or a zero residual)
    int iters;      // iterations done
    int max_iter;
    int pad;
    unsigned long long knorm_bits;  // ||K||_inf as the bits of a non-negative double
    double rnorm2, xnorm2, bnorm2, rinf;  // residual of the recovered solution
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum in a fixed order (wave sums, then the waves in order); result in every thread.
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    return s;
}

// Sum of partial column t over the G blocks of the previous kernel (every thread, fixed order).
__device__ double reduce_part(const double *part, int G, int t) {
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += part[b * 4 + t];
    return s;
}

// H_gamma entries, and the values of J and J^T gathered from K's CSR values; K's values kept
// for the residual.  Entry e of H_gamma: s = sum over its pairs (J(r,i), J(r,j)) in ascending r
// of J(r,i) * J(r,j); value = (H + D)(i,j) + gamma * s, each operation rounded.
__global__ void k_hy_ingest(int64_t nh, const int64_t *__restrict__ hd_src, const int64_t *__restrict__ pair_ptr,
                            const int64_t *__restrict__ pair_a, const int64_t *__restrict__ pair_b, double gamma,
                            const double *__restrict__ v, double *__restrict__ hval, int64_t nj,
                            const int64_t *__restrict__ jsrc, double *__restrict__ jval, int64_t njt,
                            const int64_t *__restrict__ jtsrc, double *__restrict__ jtval, int64_t nnz,
                            double *__restrict__ kval, unsigned int *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t e = t0; e < nh; e += stride) {
        double s = 0.0;
        for (int64_t q = pair_ptr[e]; q < pair_ptr[e + 1]; ++q) {
            const double prod = v[pair_a[q]] * v[pair_b[q]];
            s = s + prod;
        }
        const double t = gamma * s;
        const int64_t h = hd_src[e];
        hval[e] = (h >= 0 ? v[h] : 0.0) + t;
    }
    for (int64_t e = t0; e < nj; e += stride) jval[e] = v[jsrc[e]];
    for (int64_t e = t0; e < njt; e += stride) jtval[e] = v[jtsrc[e]];
    bool nonfinite = false;
    for (int64_t e = t0; e < nnz; e += stride) {
        kval[e] = v[e];
        nonfinite |= !isfinite(v[e]);
    }
    if (nonfinite) atomicOr(bad, 1u);
}

// out[i] = add[i] + alpha * sum_r JT(i, r) x[r] (add may be null: 0; the sum in ascending r,
// then the product by alpha, then the addition).  Returns at once when *stop is set.
__global__ void k_hy_jt(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                        const double *__restrict__ val, const double *__restrict__ x, double alpha,
                        const double *add, double *out, const int *stop) {
    if (stop && *stop) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const double prod = val[p] * x[ci[p]];
            s = s + prod;
        }
        const double t = alpha * s;
        out[i] = add ? add[i] + t : t;
    }
}

// q = J t (m rows); with sub: q = J t - sub and the CG start (r = p = q, lam = 0, partial r.r);
// without: partial p.q.  Returns at once when *stop is set.
__global__ void __launch_bounds__(kBlock) k_hy_j(int64_t m, const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ val,
                                                 const double *__restrict__ t, const double *sub, double *q,
                                                 double *r, double *p, double *lam, double *part, const int *stop) {
    __shared__ double red[kBlock / 64];
    if (!sub && *stop) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        double s = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const double prod = val[e] * t[ci[e]];
            s = s + prod;
        }
        if (sub) {
            const double c = s - sub[i];
            r[i] = c;
            p[i] = c;
            lam[i] = 0.0;
            acc += c * c;
        } else {
            q[i] = s;
            acc += p[i] * s;
        }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x * 4] = acc;
}

// CG start: rr0 = r.r from the partials; the stop threshold.
__global__ void k_hy_cg_start(int G, const double *part, double tol, int max_iter, CgControl *c) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rr = reduce_part(part, G, 0);
    c->rr = rr;
    c->rr0 = rr;
    c->tol2 = tol * tol * rr;
    c->iters = 0;
    c->max_iter = max_iter;
    c->stop = (rr == 0.0 || max_iter <= 0) ? 1 : 0;
}

// alpha = rr / (p.q); lam += alpha p; r -= alpha q; partial r.r (into the other buffer).
__global__ void __launch_bounds__(kBlock) k_hy_cg_update(int64_t m, int G, const double *part_in, double *part_out,
                                                         const double *p, const double *q, double *r, double *lam,
                                                         const CgControl *c) {
    __shared__ double red[kBlock / 64];
    if (c->stop) return;
    const double pq = reduce_part(part_in, G, 0);
    const double alpha = c->rr / pq;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        lam[i] = lam[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part_out[blockIdx.x * 4] = acc;
}

// rr' = r.r; beta = rr' / rr; p = r + beta p.  Every block reads rr from the previous launch;
// block 0 parks rr' in rr_new, which no block of this launch reads.
__global__ void __launch_bounds__(kBlock) k_hy_cg_direction(int64_t m, int G, const double *part, const double *r,
                                                            double *p, CgControl *c) {
    if (c->stop) return;
    const double rr_new = reduce_part(part, G, 0);
    const double beta = rr_new / c->rr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = r[i] + beta * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) c->rr_new = rr_new;
}

// Finishes an iteration (one thread): the new rr and the stop test.
__global__ void k_hy_cg_finish(CgControl *c) {
    if (c->stop) return;
    c->rr = c->rr_new;
    c->iters += 1;
    if (c->rr <= c->tol2 || c->iters >= c->max_iter) c->stop = 1;
}

// ||K||_inf (row absolute sums, the maximum over blocks by an atomic on its bits).
__global__ void __launch_bounds__(kBlock) k_hy_rownorm(int64_t N, const int64_t *__restrict__ rp,
                                                       const double *__restrict__ kval, CgControl *c) {
    __shared__ double red[kBlock / 64];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += fabs(kval[p]);
        m = fmax(m, s);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, red[w]);
        if (m > 0.0) atomicMax(&c->knorm_bits, __double_as_longlong(m));
    }
}

// x = [dx; lam]; rho = b - K x (row sums in CSR order); partials of ||rho||^2, ||x||^2,
// ||b||^2 and max |rho_i| (for the recovered solution's NRBE, eq. (nbre)).
__global__ void __launch_bounds__(kBlock) k_hy_resid(int64_t N, int64_t n, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const double *__restrict__ kval,
                                                     const double *dx, const double *lam, const double *b,
                                                     double *x, double *part) {
    __shared__ double red[kBlock / 64];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        x[i] = i < n ? dx[i] : lam[i - n];
    double sr = 0.0, sx = 0.0, sb = 0.0, mr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t c = ci[p];
            const double xc = c < n ? dx[c] : lam[c - n];
            const double prod = kval[p] * xc;
            s = s + prod;
        }
        const double ri = b[i] - s;
        const double xi = i < n ? dx[i] : lam[i - n];
        sr += ri * ri;
        sx += xi * xi;
        sb += b[i] * b[i];
        mr = fmax(mr, fabs(ri));
    }
    sr = block_sum(sr, red);
    sx = block_sum(sx, red);
    sb = block_sum(sb, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = sr;
        part[blockIdx.x * 4 + 1] = sx;
        part[blockIdx.x * 4 + 2] = sb;
    }
    // the max in a second pass over the wave maxima
    for (int o = 32; o > 0; o >>= 1) mr = fmax(mr, __shfl_xor(mr, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, red[w]);
        part[blockIdx.x * 4 + 3] = m;
    }
}

__global__ void k_hy_resid_reduce(int G, const double *part, CgControl *c) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double mr = 0.0;
    for (int b = 0; b < G; ++b) mr = fmax(mr, part[b * 4 + 3]);
    c->rnorm2 = reduce_part(part, G, 0);
    c->xnorm2 = reduce_part(part, G, 1);
    c->bnorm2 = reduce_part(part, G, 2);
    c->rinf = mr;
}

int grid_for(int64_t rows) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((rows + kBlock - 1) / kBlock, kGridMax));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

thread_local std::string g_hy_error;

}  // namespace

struct kkt_hykkt_s {
    kkt_hykkt_opts_t opts{};
    int64_t N = 0, n = 0, m = 0, nnz = 0;
    double gamma = 0.0;
    std::vector<int64_t> krp;
    std::vector<int32_t> kci;
    // H_gamma pattern and the map from K's values
    std::vector<int64_t> hrp, hd_src, pair_ptr, pair_a, pair_b;
    std::vector<int32_t> hci;
    // J (m x n) and J^T (n x m) in CSR with the K index of every entry
    std::vector<int64_t> jrp, jsrc, jtrp, jtsrc;
    std::vector<int32_t> jci, jtci;
    kkt_handle_t lu = nullptr;  // the H_gamma factorization
    std::string err;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false, have_factors = false;
    struct Dev {
        int64_t *krp, *hd_src, *pair_ptr, *pair_a, *pair_b, *jrp, *jsrc, *jtrp, *jtsrc;
        int32_t *kci, *jci, *jtci;
        double *kval, *hval, *jval, *jtval;
        double *rhat, *y, *u, *t, *w, *dx, *r, *p, *q, *lam, *part;
        CgControl *ctl;
        unsigned int *bad;
    } d{};
    CgControl *host_ctl = nullptr;  // pinned copy read by the host
};

namespace {

kkt_status_t hy_fail(kkt_hykkt_t h, kkt_status_t s, const std::string &m) {
    if (h) h->err = m;
    g_hy_error = m;
    return s;
}

#define HY_HIP(h, call)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return hy_fail((h), KKT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Byte offsets of the HyKKT arrays in the workspace (the H_gamma factorization's workspace
// follows at `lu`).
struct HyPlan {
    size_t krp, kci, kval, hd_src, pair_ptr, pair_a, pair_b, hval, jrp, jci, jsrc, jval, jtrp, jtci, jtsrc, jtval,
        rhat, y, u, t, w, dx, r, p, q, lam, part, ctl, bad, lu, lu_bytes, total;
};

HyPlan hy_plan(const kkt_hykkt_t h) {
    HyPlan o{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t nh = h->hci.size(), np = h->pair_a.size();
    o.krp = take(8 * (h->N + 1));
    o.kci = take(4 * h->nnz);
    o.kval = take(8 * h->nnz);
    o.hd_src = take(8 * nh);
    o.pair_ptr = take(8 * (nh + 1));
    o.pair_a = take(8 * np);
    o.pair_b = take(8 * np);
    o.hval = take(8 * nh);
    o.jrp = take(8 * (h->m + 1));
    o.jci = take(4 * h->jci.size());
    o.jsrc = take(8 * h->jsrc.size());
    o.jval = take(8 * h->jsrc.size());
    o.jtrp = take(8 * (h->n + 1));
    o.jtci = take(4 * h->jtci.size());
    o.jtsrc = take(8 * h->jtsrc.size());
    o.jtval = take(8 * h->jtsrc.size());
    for (size_t *v : {&o.rhat, &o.y, &o.u, &o.t, &o.w, &o.dx}) *v = take(8 * h->n);
    for (size_t *v : {&o.r, &o.p, &o.q, &o.lam}) *v = take(8 * h->m);
    o.part = take(8 * 2 * 4 * kGridMax);
    o.ctl = take(sizeof(CgControl));
    o.bad = take(sizeof(unsigned int));
    size_t lub = 0;
    kkt_workspace_size(h->lu, 1, &lub);
    o.lu = take(0);
    o.lu_bytes = lub;
    o.total = align256(o.lu + lub);
    return o;
}

template <typename T> hipError_t up(char *base, size_t off, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

extern "C" {

void kkt_hykkt_opts_default(kkt_hykkt_opts_t *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->gamma = 0.0;
    o->gamma_scale = 1e4;
    o->cg_tol = 1e-12;
    o->cg_max_iter = 1000;
    kkt_opts_default(&o->lu);
}

kkt_status_t kkt_hykkt_analyze(const kkt_hykkt_opts_t *opts, int64_t N, int64_t n_primal, const int64_t *rowptr,
                               const int32_t *colidx, const double *values_first, kkt_hykkt_t *out) {
    if (!out) return hy_fail(nullptr, KKT_EINVAL, "null output handle");
    *out = nullptr;
    if (!rowptr || !colidx || !values_first) return hy_fail(nullptr, KKT_EINVAL, "null argument");
    if (N < 2 || n_primal < 1 || n_primal >= N) return hy_fail(nullptr, KKT_EINVAL, "need 1 <= n_primal < N");
    kkt_hykkt_t h = new (std::nothrow) kkt_hykkt_s();
    if (!h) return hy_fail(nullptr, KKT_ENOMEM, "out of host memory");
    try {
        if (opts) h->opts = *opts;
        else kkt_hykkt_opts_default(&h->opts);
        if (!(h->opts.cg_tol > 0.0) || h->opts.cg_max_iter < 1 || h->opts.gamma < 0.0 ||
            (h->opts.gamma == 0.0 && !(h->opts.gamma_scale > 0.0))) {
            delete h;
            return hy_fail(nullptr, KKT_EINVAL, "invalid HyKKT options");
        }
        const int64_t n = n_primal, m = N - n_primal;
        h->N = N;
        h->n = n;
        h->m = m;
        h->nnz = rowptr[N];
        if (rowptr[0] != 0 || h->nnz < 1) {
            delete h;
            return hy_fail(nullptr, KKT_EINVAL, "bad row pointers");
        }
        h->krp.assign(rowptr, rowptr + N + 1);
        h->kci.assign(colidx, colidx + h->nnz);
        for (int64_t i = 0; i < N; ++i) {
            if (rowptr[i + 1] < rowptr[i]) {
                delete h;
                return hy_fail(nullptr, KKT_EINVAL, "row pointers decrease");
            }
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                if (colidx[p] < 0 || colidx[p] >= N || (p > rowptr[i] && colidx[p] <= colidx[p - 1])) {
                    delete h;
                    return hy_fail(nullptr, KKT_EINVAL, "columns out of range, unsorted or repeated in row " +
                                                            std::to_string(i));
                }
                if (!std::isfinite(values_first[p])) {
                    delete h;
                    return hy_fail(nullptr, KKT_EINVAL, "non-finite value");
                }
                if (i >= n && colidx[p] >= n && values_first[p] != 0.0) {
                    delete h;
                    return hy_fail(nullptr, KKT_EINVAL, "HyKKT needs a zero (2,2) block (row " + std::to_string(i) + ")");
                }
            }
        }
        // J rows (K rows n.., columns < n) and J^T rows (K rows < n, columns >= n)
        h->jrp.assign(m + 1, 0);
        for (int64_t r = 0; r < m; ++r) {
            for (int64_t p = rowptr[n + r]; p < rowptr[n + r + 1]; ++p)
                if (colidx[p] < n) {
                    h->jci.push_back(colidx[p]);
                    h->jsrc.push_back(p);
                }
            h->jrp[r + 1] = (int64_t)h->jci.size();
        }
        h->jtrp.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (colidx[p] >= n) {
                    h->jtci.push_back((int32_t)(colidx[p] - n));
                    h->jtsrc.push_back(p);
                }
            h->jtrp[i + 1] = (int64_t)h->jtci.size();
        }
        // gamma from system 1 (the rule: scale * max_i A_ii / max_i (J^T J)_ii)
        const double *v = values_first;
        if (h->opts.gamma > 0.0) {
            h->gamma = h->opts.gamma;
        } else {
            double amax = 0.0;
            for (int64_t i = 0; i < n; ++i)
                for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                    if (colidx[p] == i) amax = std::max(amax, v[p]);
            std::vector<double> jtj(n, 0.0);
            for (int64_t r = 0; r < m; ++r)
                for (int64_t e = h->jrp[r]; e < h->jrp[r + 1]; ++e) {
                    const double x = v[h->jsrc[e]];
                    const double prod = x * x;
                    jtj[h->jci[e]] = jtj[h->jci[e]] + prod;
                }
            const double jmax = *std::max_element(jtj.begin(), jtj.end());
            if (!(jmax > 0.0) || !(amax > 0.0)) {
                delete h;
                return hy_fail(nullptr, KKT_EINVAL, "HyKKT needs a nonzero J and a positive diagonal of H + D");
            }
            h->gamma = h->opts.gamma_scale * amax / jmax;
        }
        // H_gamma pattern and map: row i = columns of A(i,:) joined with those of J(r,:) for the
        // constraint rows r touching column i (ascending r)
        std::vector<std::vector<int64_t>> col_rows(n);
        for (int64_t r = 0; r < m; ++r)
            for (int64_t e = h->jrp[r]; e < h->jrp[r + 1]; ++e) col_rows[h->jci[e]].push_back(r);
        std::vector<int64_t> where(n, -1);   // column -> K index of A(i, col) for the current row
        std::vector<int64_t> jwhere(n, -1);  // column -> entry of J(r, col) for the current r
        h->hrp.assign(n + 1, 0);
        h->pair_ptr.push_back(0);
        std::vector<int32_t> cols;
        for (int64_t i = 0; i < n; ++i) {
            cols.clear();
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (colidx[p] < n) {
                    where[colidx[p]] = p;
                    cols.push_back(colidx[p]);
                }
            for (int64_t r : col_rows[i])
                for (int64_t e = h->jrp[r]; e < h->jrp[r + 1]; ++e) cols.push_back(h->jci[e]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int32_t j : cols) {
                h->hci.push_back(j);
                h->hd_src.push_back(where[j]);
                for (int64_t r : col_rows[i]) {  // ascending r
                    int64_t ei = -1, ej = -1;
                    for (int64_t e = h->jrp[r]; e < h->jrp[r + 1]; ++e) {
                        if (h->jci[e] == i) ei = e;
                        if (h->jci[e] == j) ej = e;
                    }
                    if (ei >= 0 && ej >= 0) {
                        h->pair_a.push_back(h->jsrc[ei]);
                        h->pair_b.push_back(h->jsrc[ej]);
                    }
                }
                h->pair_ptr.push_back((int64_t)h->pair_a.size());
            }
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (colidx[p] < n) where[colidx[p]] = -1;
            h->hrp[i + 1] = (int64_t)h->hci.size();
        }
        (void)jwhere;
        // system 1's H_gamma values (same operations as k_hy_ingest) and its analysis
        const size_t nh = h->hci.size();
        std::vector<double> hv(nh);
        for (size_t e = 0; e < nh; ++e) {
            double s = 0.0;
            for (int64_t q = h->pair_ptr[e]; q < h->pair_ptr[e + 1]; ++q) {
                const double prod = v[h->pair_a[q]] * v[h->pair_b[q]];
                s = s + prod;
            }
            const double t = h->gamma * s;
            hv[e] = (h->hd_src[e] >= 0 ? v[h->hd_src[e]] : 0.0) + t;
        }
        const kkt_status_t st = kkt_analyze(&h->opts.lu, n, h->hrp.data(), h->hci.data(), hv.data(), &h->lu);
        if (st != KKT_OK) {
            const std::string msg = std::string("H_gamma analysis: ") + kkt_last_error(nullptr);
            delete h;
            return hy_fail(nullptr, st, msg);
        }
    } catch (const std::bad_alloc &) {
        delete h;
        return hy_fail(nullptr, KKT_ENOMEM, "out of host memory");
    }
    *out = h;
    return KKT_OK;
}

kkt_status_t kkt_hykkt_workspace_size(kkt_hykkt_t h, size_t *bytes) {
    if (!h || !bytes) return hy_fail(h, KKT_EINVAL, "null argument");
    *bytes = hy_plan(h).total;
    return KKT_OK;
}

kkt_status_t kkt_hykkt_bind_workspace(kkt_hykkt_t h, void *dev_ptr, size_t bytes, void *stream) {
    if (!h) return hy_fail(h, KKT_EINVAL, "null handle");
    const HyPlan o = hy_plan(h);
    if (!dev_ptr || bytes < o.total) return hy_fail(h, KKT_ENOMEM, "workspace too small");
    if (((uintptr_t)dev_ptr & 255) != 0) return hy_fail(h, KKT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)dev_ptr;
    auto &d = h->d;
    d.krp = (int64_t *)(b + o.krp);
    d.kci = (int32_t *)(b + o.kci);
    d.kval = (double *)(b + o.kval);
    d.hd_src = (int64_t *)(b + o.hd_src);
    d.pair_ptr = (int64_t *)(b + o.pair_ptr);
    d.pair_a = (int64_t *)(b + o.pair_a);
    d.pair_b = (int64_t *)(b + o.pair_b);
    d.hval = (double *)(b + o.hval);
    d.jrp = (int64_t *)(b + o.jrp);
    d.jci = (int32_t *)(b + o.jci);
    d.jsrc = (int64_t *)(b + o.jsrc);
    d.jval = (double *)(b + o.jval);
    d.jtrp = (int64_t *)(b + o.jtrp);
    d.jtci = (int32_t *)(b + o.jtci);
    d.jtsrc = (int64_t *)(b + o.jtsrc);
    d.jtval = (double *)(b + o.jtval);
    d.rhat = (double *)(b + o.rhat);
    d.y = (double *)(b + o.y);
    d.u = (double *)(b + o.u);
    d.t = (double *)(b + o.t);
    d.w = (double *)(b + o.w);
    d.dx = (double *)(b + o.dx);
    d.r = (double *)(b + o.r);
    d.p = (double *)(b + o.p);
    d.q = (double *)(b + o.q);
    d.lam = (double *)(b + o.lam);
    d.part = (double *)(b + o.part);
    d.ctl = (CgControl *)(b + o.ctl);
    d.bad = (unsigned int *)(b + o.bad);
    HY_HIP(h, up(b, o.krp, h->krp, s));
    HY_HIP(h, up(b, o.kci, h->kci, s));
    HY_HIP(h, up(b, o.hd_src, h->hd_src, s));
    HY_HIP(h, up(b, o.pair_ptr, h->pair_ptr, s));
    HY_HIP(h, up(b, o.pair_a, h->pair_a, s));
    HY_HIP(h, up(b, o.pair_b, h->pair_b, s));
    HY_HIP(h, up(b, o.jrp, h->jrp, s));
    HY_HIP(h, up(b, o.jci, h->jci, s));
    HY_HIP(h, up(b, o.jsrc, h->jsrc, s));
    HY_HIP(h, up(b, o.jtrp, h->jtrp, s));
    HY_HIP(h, up(b, o.jtci, h->jtci, s));
    HY_HIP(h, up(b, o.jtsrc, h->jtsrc, s));
    HY_HIP(h, hipMemsetAsync(d.ctl, 0, sizeof(CgControl), s));
    HY_HIP(h, hipStreamSynchronize(s));
    if (!h->host_ctl) HY_HIP(h, hipHostMalloc((void **)&h->host_ctl, sizeof(CgControl), hipHostMallocDefault));
    const kkt_status_t st = kkt_bind_workspace(h->lu, b + o.lu, o.lu_bytes, stream);
    if (st != KKT_OK) return hy_fail(h, st, std::string("H_gamma workspace: ") + kkt_last_error(h->lu));
    h->ws = b;
    h->ws_bytes = bytes;
    h->bound = true;
    h->have_factors = false;
    return KKT_OK;
}

kkt_status_t kkt_hykkt_refactor(kkt_hykkt_t h, const double *dev_values, void *stream) {
    if (!h || !dev_values) return hy_fail(h, KKT_EINVAL, "null argument");
    if (!h->bound) return hy_fail(h, KKT_ESTATE, "no workspace bound");
    hipStream_t s = (hipStream_t)stream;
    auto &d = h->d;
    HY_HIP(h, hipMemsetAsync(d.bad, 0, sizeof(unsigned int), s));
    HY_HIP(h, hipMemsetAsync(&d.ctl->knorm_bits, 0, sizeof(unsigned long long), s));
    k_hy_ingest<<<2048, kBlock, 0, s>>>((int64_t)h->hci.size(), d.hd_src, d.pair_ptr, d.pair_a, d.pair_b, h->gamma,
                                        dev_values, d.hval, (int64_t)h->jsrc.size(), d.jsrc, d.jval,
                                        (int64_t)h->jtsrc.size(), d.jtsrc, d.jtval, h->nnz, d.kval, d.bad);
    k_hy_rownorm<<<grid_for(h->N), kBlock, 0, s>>>(h->N, d.krp, d.kval, d.ctl);
    HY_HIP(h, hipGetLastError());
    const kkt_status_t st = kkt_refactor(h->lu, d.hval, stream);
    if (st != KKT_OK) return hy_fail(h, st, std::string("H_gamma refactorization: ") + kkt_last_error(h->lu));
    h->have_factors = true;
    return KKT_OK;
}

kkt_status_t kkt_hykkt_solve(kkt_hykkt_t h, const double *dev_b, double *dev_x, kkt_hykkt_info_t *info,
                             void *stream) {
    if (!h || !dev_b || !dev_x) return hy_fail(h, KKT_EINVAL, "null argument");
    if (dev_b == dev_x) return hy_fail(h, KKT_EINVAL, "b and x must be distinct");
    if (!h->bound || !h->have_factors) return hy_fail(h, KKT_ESTATE, "refactor before solve");
    hipStream_t s = (hipStream_t)stream;
    auto &d = h->d;
    const int64_t n = h->n, m = h->m;
    const int gn = grid_for(n), gm = grid_for(m), gN = grid_for(h->N);
    double *partA = d.part, *partB = d.part + 4 * kGridMax;
    const double *bx = dev_b, *bl = dev_b + n;
    auto hinv = [&](const double *in, double *outv) -> kkt_status_t {
        const kkt_status_t st = kkt_direct_solve(h->lu, in, outv, stream);
        return st == KKT_OK ? st : hy_fail(h, st, std::string("H_gamma solve: ") + kkt_last_error(h->lu));
    };
    // rhat = r_x + gamma J^T r_l;  y = H_gamma^-1 rhat;  c = J y - r_l  (r = p = c, lam = 0)
    k_hy_jt<<<gn, kBlock, 0, s>>>(n, d.jtrp, d.jtci, d.jtval, bl, h->gamma, bx, d.rhat, nullptr);
    kkt_status_t st = hinv(d.rhat, d.y);
    if (st != KKT_OK) return st;
    k_hy_j<<<gm, kBlock, 0, s>>>(m, d.jrp, d.jci, d.jval, d.y, bl, nullptr, d.r, d.p, d.lam, partA, nullptr);
    k_hy_cg_start<<<1, 64, 0, s>>>(gm, partA, h->opts.cg_tol, h->opts.cg_max_iter, d.ctl);
    HY_HIP(h, hipGetLastError());
    const int *stop = &d.ctl->stop;
    for (;;) {
        for (int k = 0; k < kCgGroup; ++k) {
            // q = S p = J H_gamma^-1 J^T p
            k_hy_jt<<<gn, kBlock, 0, s>>>(n, d.jtrp, d.jtci, d.jtval, d.p, 1.0, nullptr, d.u, stop);
            st = hinv(d.u, d.t);
            if (st != KKT_OK) return st;
            k_hy_j<<<gm, kBlock, 0, s>>>(m, d.jrp, d.jci, d.jval, d.t, nullptr, d.q, d.r, d.p, d.lam, partA, stop);
            k_hy_cg_update<<<gm, kBlock, 0, s>>>(m, gm, partA, partB, d.p, d.q, d.r, d.lam, d.ctl);
            k_hy_cg_direction<<<gm, kBlock, 0, s>>>(m, gm, partB, d.r, d.p, d.ctl);
            k_hy_cg_finish<<<1, 1, 0, s>>>(d.ctl);
        }
        HY_HIP(h, hipGetLastError());
        HY_HIP(h, hipMemcpyAsync(h->host_ctl, d.ctl, sizeof(CgControl), hipMemcpyDeviceToHost, s));
        HY_HIP(h, hipStreamSynchronize(s));
        if (h->host_ctl->stop) break;
    }
    const CgControl cg = *h->host_ctl;
    // dx = H_gamma^-1 (rhat - J^T lam);  x = [dx; lam] and its residual in K
    k_hy_jt<<<gn, kBlock, 0, s>>>(n, d.jtrp, d.jtci, d.jtval, d.lam, -1.0, d.rhat, d.w, nullptr);
    st = hinv(d.w, d.dx);
    if (st != KKT_OK) return st;
    k_hy_resid<<<gN, kBlock, 0, s>>>(h->N, n, d.krp, d.kci, d.kval, d.dx, d.lam, dev_b, dev_x, partA);
    k_hy_resid_reduce<<<1, 64, 0, s>>>(gN, partA, d.ctl);
    HY_HIP(h, hipGetLastError());
    HY_HIP(h, hipMemcpyAsync(h->host_ctl, d.ctl, sizeof(CgControl), hipMemcpyDeviceToHost, s));
    unsigned int bad = 0;
    HY_HIP(h, hipMemcpyAsync(&bad, d.bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HY_HIP(h, hipStreamSynchronize(s));
    if (bad) return hy_fail(h, KKT_EINVAL, "non-finite value in K");
    const CgControl &c = *h->host_ctl;
    const double rn = std::sqrt(c.rnorm2), xn = std::sqrt(c.xnorm2), bn = std::sqrt(c.bnorm2);
    double knorm = 0.0;
    std::memcpy(&knorm, &c.knorm_bits, sizeof(double));
    const bool converged = cg.rr <= cg.tol2;
    if (info) {
        info->converged = converged ? 1 : 0;
        info->cg_iterations = cg.iters;
        info->gamma = h->gamma;
        info->cg_rel_resid = cg.rr0 > 0.0 ? std::sqrt(cg.rr / cg.rr0) : 0.0;
        info->true_resid = rn;
        info->knorm_inf = knorm;
        info->nrbe = rn / (knorm * xn + bn);
        info->rel_resid = bn > 0.0 ? rn / bn : 0.0;
    }
    return converged ? KKT_OK : hy_fail(h, KKT_ENOCONV, "CG reached its iteration cap");
}

kkt_status_t kkt_hykkt_get_hgamma(kkt_hykkt_t h, int64_t *rp, int32_t *ci, double *vals, double *gamma, void *stream) {
    if (!h) return hy_fail(h, KKT_EINVAL, "null handle");
    if (rp) std::memcpy(rp, h->hrp.data(), h->hrp.size() * sizeof(int64_t));
    if (ci) std::memcpy(ci, h->hci.data(), h->hci.size() * sizeof(int32_t));
    if (gamma) *gamma = h->gamma;
    if (vals) {
        if (!h->have_factors) return hy_fail(h, KKT_ESTATE, "no values before a refactorization");
        HY_HIP(h, hipMemcpyAsync(vals, h->d.hval, h->hci.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 (hipStream_t)stream));
        HY_HIP(h, hipStreamSynchronize((hipStream_t)stream));
    }
    return KKT_OK;
}

kkt_status_t kkt_hykkt_sizes(kkt_hykkt_t h, int64_t *nnz_hgamma, int64_t *pairs) {
    if (!h) return hy_fail(h, KKT_EINVAL, "null handle");
    if (nnz_hgamma) *nnz_hgamma = (int64_t)h->hci.size();
    if (pairs) *pairs = (int64_t)h->pair_a.size();
    return KKT_OK;
}

kkt_status_t kkt_hykkt_factor_handle(kkt_hykkt_t h, kkt_handle_t *lu) {
    if (!h || !lu) return hy_fail(h, KKT_EINVAL, "null argument");
    *lu = h->lu;
    return KKT_OK;
}

const char *kkt_hykkt_last_error(kkt_hykkt_t h) { return h ? h->err.c_str() : g_hy_error.c_str(); }

kkt_status_t kkt_hykkt_release(kkt_hykkt_t h) {
    if (!h) return KKT_OK;
    if (h->lu) kkt_release(h->lu);
    if (h->host_ctl) (void)hipHostFree(h->host_ctl);
    delete h;
    return KKT_OK;
}

}  // extern "C"
