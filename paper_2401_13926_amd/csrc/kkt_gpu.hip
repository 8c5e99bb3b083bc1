// GPU refactorization, triangular solves and FGMRES-IR for sequences of sparse KKT systems on
// MI355X (gfx950), and the C ABI declared in include/kkt.h.
//
// Paper: Swirydowicz et al., "Iterative Methods in GPU-Resident Linear Solvers for Nonlinear
// Constrained Optimization".  Section 1.3: refactorization with static pivoting; Section 2.1:
// FGMRES iterative refinement with the LU factors as right preconditioner and CGS2;
// Section 2.2: NRBE (eq. (nbre)); Section 2.3: the refine decision.
//
// Kernels (all wave64):
//   k_ingest_rows / k_arm    new values -> the solve's copy of K, ||K||_inf, finiteness;
//                            sentinels (and, without the flat list, the factor storage)
//   k_refactor<T>            eager left-looking numeric LU, one wavefront per column, columns
//                            handed out in dependency-level order; a column starts its update
//                            chain at once and waits per entry of each source column (every
//                            finished L entry is its own ready flag, so no memory fences)
//   k_trsv<T, LOWER>         row-oriented triangular solve by tiles (a block walks the
//                            segments of its tile, g lanes per row); a solution entry is its
//                            own ready flag (a NaN sentinel until written)
//   k_spmv_dots, k_cgs_*, k_normalize, k_resid, k_xupdate   Krylov kernels; block partial
//                            sums are reduced by the next kernel in fixed order (deterministic,
//                            no fences)
//
// Floating point: compiled with -ffp-contract=off, so the refactorization performs exactly
// the roundings of a left-looking column LU with ascending updates (reproducible factors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "analysis.hpp"
#include "kernels.hpp"

namespace kkt {

// ---------------------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------------------

// Sentinels: signalling-NaN bit patterns no arithmetic result can take.
constexpr unsigned long long kSent64 = 0x7FF4DEADBEEF0001ull;
constexpr unsigned int kSent32 = 0x7FA0BEEFu;

template <typename T> struct Bits;
template <> struct Bits<double> {
    using U = unsigned long long;
    static constexpr U sent = kSent64;
};
template <> struct Bits<float> {
    using U = unsigned int;
    static constexpr U sent = kSent32;
};

template <typename T> __device__ __forceinline__ T sentinel() {
    return __builtin_bit_cast(T, Bits<T>::sent);
}
template <typename T> __device__ __forceinline__ bool is_sentinel(T v) {
    return __builtin_bit_cast(typename Bits<T>::U, v) == Bits<T>::sent;
}

// Ready-flag values are published and polled at system scope: on a multi-XCD device a
// device-scope store can sit in the producer XCD's L2 until that line is evicted (observed:
// about a millisecond), while system-scope accesses go through to memory.
template <typename T> __device__ __forceinline__ void store_ready(T *p, T v) {
    using U = typename Bits<T>::U;
    __hip_atomic_store(reinterpret_cast<U *>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// Value of a solution entry produced by another wavefront: a plain load first (it can only
// return the sentinel or the final value), then coherent polling until it is written.  A
// wait longer than kSpinLimit sets *hang and gives up (every later wait then returns at
// once), so a broken schedule ends the kernel with an error instead of never finishing.
// Waits until *p no longer holds the sentinel.  kInFlight = 4: four coherent loads in
// flight, one issued per check, so a store is seen about a quarter of a memory round trip
// after it lands (the refactorization's waits, which sit on its critical chain).
// kInFlight = 1: one load at a time (the triangular solves' staging waits, which overlap
// other tiles' loads: less polling traffic measured faster there).
template <typename T, int kInFlight = 4, int kSleep = 1>
__device__ __forceinline__ T load_ready(const T *p, unsigned int *hang) {
    static_assert(kInFlight == 4 || kInFlight == 1, "4 or 1 loads in flight");
    using U = typename Bits<T>::U;
    T v = *p;
    if (!is_sentinel(v)) return v;
    const U *q = reinterpret_cast<const U *>(p);
    unsigned int spins = 0;
    if (kInFlight == 1) {
        // (no early exit on another wave's hang flag: the check measured slower in this loop;
        // every waiting lane still gives up after kSpinLimit polls)
        for (;;) {
            const U b = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (b != Bits<T>::sent) return __builtin_bit_cast(T, b);
            if (++spins >= kSpinLimit) {
                __hip_atomic_store(hang, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return T(0);
            }
            __builtin_amdgcn_s_sleep(kSleep);
        }
    }
    U b0 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_s_sleep(1);
    U b1 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_s_sleep(1);
    U b2 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_s_sleep(1);
    U b3 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (;;) {
        if (b0 != Bits<T>::sent) return __builtin_bit_cast(T, b0);
        b0 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (b1 != Bits<T>::sent) return __builtin_bit_cast(T, b1);
        b1 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (b2 != Bits<T>::sent) return __builtin_bit_cast(T, b2);
        b2 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (b3 != Bits<T>::sent) return __builtin_bit_cast(T, b3);
        b3 = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        spins += 4;
        if (spins >= kSpinLimit ||
            ((spins & 1023u) == 0 && __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
            __hip_atomic_store(hang, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return T(0);
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Wave-uniform: lane 0 takes `chunk` consecutive work items from *counter.
__device__ __forceinline__ unsigned int grab(unsigned int *counter, unsigned int chunk) {
    unsigned int v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(counter, chunk);
    return __shfl(v, 0, 64);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide sum of one double per thread (blockDim = kStreamBlock); result in all threads.
__device__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kStreamBlock / 64; ++w) s += red[w];
    return s;
}

// Block-wide max of non-negative doubles (blockDim = kStreamBlock); result in all threads.
__device__ double block_max(double v, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kStreamBlock / 64; ++w) s = fmax(s, red[w]);
    return s;
}

// Row range of block b when `total` rows are split into gridDim.x contiguous chunks.
__device__ __forceinline__ void block_rows(int64_t total, int64_t &r0, int64_t &r1) {
    const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
    r0 = (int64_t)blockIdx.x * chunk;
    r1 = r0 + chunk < total ? r0 + chunk : total;
}

// ---------------------------------------------------------------------------------------
// ingest: K values into the workspace and into the factor layout (fill entries = 0)
// ---------------------------------------------------------------------------------------

__global__ void k_prep_solve(Control *c) {
    c->hang = 0;
    c->nonfinite_b = 0;
    c->counter = 0;
    c->stop = 0;
}

// Before the values of a new system: the row-norm maximum and the finiteness flag.
__global__ void k_prep_values(Control *c) {
    c->knorm_bits = 0;
    c->nonfinite = 0;
}

// Before a refactorization (of new values or of the ones already ingested).
__global__ void k_prep_refactor(Control *c) {
    for (int q = 0; q < kWorkQueues; ++q) c->work_refactor[q * 64] = 0;
    c->hang = 0;
    c->guard_fail = 0;
    c->nguard = 0;
    c->counter = 0;
}

// New values: K's values (original CSR order, vals) into the Krylov side's copy in the vector
// order, one thread per row of the copy (row k is an original row whose entries start at
// ostart[k] and keep their order); also ||K||_inf (each row's absolute values summed in
// order, one atomic maximum per block) and the finiteness of every value.
__global__ void k_ingest_rows(int64_t n, const int64_t *__restrict__ ostart, const int64_t *__restrict__ krp,
                              const double *__restrict__ vals, double *__restrict__ kval, Control *c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double m = 0.0;
    bool bad = false;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int64_t s = ostart[k], e0 = krp[k];
        const int len = (int)(krp[k + 1] - e0);
        double sum = 0.0;
        for (int t0 = 0; t0 < len; t0 += 8) {
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = t0 + t < len ? vals[s + t0 + t] : 0.0;
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (t0 + t < len) {
                    kval[e0 + t0 + t] = v[t];
                    sum += fabs(v[t]);
                    bad |= !isfinite(v[t]);
                }
        }
        m = fmax(m, sum);
    }
    // one atomic per block: atomics on one address serialize
    __shared__ double red[256 / 64];
    __shared__ int redb[256 / 64];
    m = wave_max(m);
    const bool wbad = __any(bad);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = m;
        redb[threadIdx.x >> 6] = wbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bool b = redb[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            m = fmax(m, red[w]);
            b = b || redb[w];
        }
        if (m > 0.0) atomicMax(&c->knorm_bits, __double_as_longlong(m));
        if (b) atomicOr(&c->nonfinite, 1u);
    }
}

// Arms the finished-value array of the refactorization with sentinels; without the flat list
// also the factor storage from the copy of K (fill = 0), which that refactorization updates in
// place (with it, the columns are staged from K's values directly).
__global__ void k_arm(int64_t f, const int64_t *__restrict__ fsrc, const double *__restrict__ kval,
                      double *__restrict__ F64, float *__restrict__ F32, double *__restrict__ Ld64,
                      float *__restrict__ Ld32, int mixed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < f; t += stride) {
        double v = 0.0;
        if (fsrc) {
            const int64_t s = fsrc[t];
            v = s >= 0 ? kval[s] : 0.0;
        }
        if (mixed) {
            if (fsrc) F32[t] = (float)v;
            Ld32[t] = sentinel<float>();
        } else {
            if (fsrc) F64[t] = v;
            Ld64[t] = sentinel<double>();
        }
    }
}

// Vectors between the caller's (original) order and the vector order of a solve:
// out[k] = in[perm[k]] (gather) and out[perm[k]] = in[k] (scatter).
__global__ void k_vgather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ in,
                          double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) out[k] = in[perm[k]];
}
__global__ void k_vscatter(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ in,
                           double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) out[perm[k]] = in[k];
}

// CSR row loops issue a row's loads kRowBatch at a time (index and value loads together, then
// the gathers), so a short row costs one round of dependent loads instead of one per entry;
// the terms are still combined one by one in ascending position.
constexpr int kRowBatch = 8;

// sum over p in [rp[i], rp[i+1]) of kval[p] * x[ci[p]], each product and sum rounded, in
// ascending p
__device__ __forceinline__ double row_dot(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                          const double *__restrict__ kval, const double *x, int64_t i) {
    const int64_t e = rp[i + 1];
    double s = 0.0;
    for (int64_t p = rp[i]; p < e; p += kRowBatch) {
        int c[kRowBatch];
        double v[kRowBatch], xv[kRowBatch];
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) {
            c[t] = p + t < e ? ci[p + t] : 0;
            v[t] = p + t < e ? kval[p + t] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) xv[t] = p + t < e ? x[c[t]] : 0.0;
#pragma unroll
        for (int t = 0; t < kRowBatch; ++t) {
            if (p + t < e) {
                const double prod = v[t] * xv[t];
                s = s + prod;
            }
        }
    }
    return s;
}

// ||K||_inf of the values already in the workspace's copy of K (after a re-pivot, which
// uploads them from the host).
__global__ void k_rownorm(int64_t n, const int64_t *__restrict__ rp, const double *__restrict__ kval,
                          Control *c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        const int64_t e = rp[i + 1];
        for (int64_t p = rp[i]; p < e; p += kRowBatch) {
            double v[kRowBatch];
#pragma unroll
            for (int t = 0; t < kRowBatch; ++t) v[t] = p + t < e ? kval[p + t] : 0.0;
#pragma unroll
            for (int t = 0; t < kRowBatch; ++t)
                if (p + t < e) s += fabs(v[t]);
        }
        m = fmax(m, s);
    }
    // one atomic per block: atomics on one address serialize (one per wavefront cost about
    // 100 us at 2M rows)
    __shared__ double red[256 / 64];
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        if (m > 0.0) atomicMax(&c->knorm_bits, __double_as_longlong(m));
    }
}

// ---------------------------------------------------------------------------------------
// refactorization (static pivots): one wavefront per column, eager left-looking
// ---------------------------------------------------------------------------------------

template <typename T> struct RefactorArgs {
    int64_t n;
    const int64_t *fp;
    const int32_t *fi;
    const int32_t *fdiag;
    const int64_t *relptr;
    const int32_t *relpos;
    const int32_t *order;
    const int32_t *clev;  // level of each order position
    const int32_t *f2t;
    const int32_t *relsrc;   // per update: F index of the L entry it applies
    const int32_t *relslot;  // per update: position of its source's U entry in the column
    // flat list only (F and the update lists stored in col_order): first F position, first
    // update (n + 1 each) and diagonal offset of the column at each col_order position
    const int64_t *pc, *pu;
    const int32_t *pnu;
    const int32_t *fsrc;   // flat list only: per F position, its value's entry in kval, or -1
    const double *kval;    // flat list only: K's values (the column staging reads them)
    const int32_t *item;     // hand-out items: first col_order position of each (nitems + 1)
    const uint8_t *item_lane;  // 1: one column per lane
    int64_t nitems;
    T *F;                // working columns of the paths that update in HBM (final values: Tv)
    T *Tv;               // solve layout copy
    T *Ld;               // finished L values in F layout; sentinel until written (ready flags)
    int guard_fail_policy;
    Control *ctl;
};

template <typename T> __device__ __forceinline__ T unit_roundoff();
template <> __device__ __forceinline__ double unit_roundoff<double>() { return 0x1p-53; }
template <> __device__ __forceinline__ float unit_roundoff<float>() { return 0x1p-24f; }

// Applies the update chain of column j (its update positions start at rp) to x (LDS or the
// column's own global storage): for each source step k of U(:,j) in ascending order,
// x[relpos] -= L(:,k) * x[k].  The values
// of L(:,k) come from the finished-value array; an entry still holding the sentinel is
// polled until its column's wavefront has written it (no fences: every entry is its own
// flag, written once with a coherent store).
template <typename T, bool kLds>
__device__ void refactor_chain(const RefactorArgs<T> &a, int64_t rp, int64_t c0, int nu, T *x) {
    const int lane = threadIdx.x & 63;
    unsigned int *hang = &a.ctl->hang;
    for (int t0 = 0; t0 < nu; t0 += 64) {
        const int cnt = nu - t0 < 64 ? nu - t0 : 64;
        // lane s holds the metadata of source step t0 + s: its L part [l0, l0 + nl)
        int64_t l0_l = 0;
        int nl_l = 0;
        if (lane < cnt) {
            const int k = a.fi[c0 + t0 + lane];
            l0_l = a.fp[k] + a.fdiag[k] + 1;
            nl_l = (int)(a.fp[k + 1] - l0_l);
        }
        // offset of each step's update positions: exclusive prefix sum of nl over lanes
        int off_l = nl_l;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(off_l, o, 64);
            if (lane >= o) off_l += v;
        }
        off_l -= nl_l;
        // first 64 updates of a step: its L values and positions are loaded two steps ahead
        // (two dependent loads in flight per lane while a step is applied)
        auto fetch = [&](int st, int64_t &l0x, int &nlx, int64_t &rox, T &lvx, int &posx) {
            l0x = 0;
            nlx = 0;
            rox = 0;
            lvx = T(0);
            posx = 0;
            if (st < cnt) {
                l0x = __shfl(l0_l, st, 64);
                nlx = __shfl(nl_l, st, 64);
                rox = rp + __shfl(off_l, st, 64);
                if (lane < nlx) {
                    lvx = a.Ld[l0x + lane];
                    posx = a.relpos[rox + lane];
                }
            }
        };
        int64_t l0, ro, l0n, ron;
        int nl, pos, nln, posn;
        T lv, lvn;
        fetch(0, l0, nl, ro, lv, pos);
        fetch(1, l0n, nln, ron, lvn, posn);
        for (int s = 0; s < cnt; ++s) {
            int64_t l0nn, ronn;
            int nlnn, posnn;
            T lvnn;
            fetch(s + 2, l0nn, nlnn, ronn, lvnn, posnn);
            if (lane < nl && is_sentinel(lv)) lv = load_ready(a.Ld + l0 + lane, hang);
            const T u = x[t0 + s];
            if (lane < nl) {
                const T prod = lv * u;
                x[pos] = x[pos] - prod;
            }
            for (int e = 64 + lane; e < nl; e += 64) {
                T lv2 = a.Ld[l0 + e];
                if (is_sentinel(lv2)) lv2 = load_ready(a.Ld + l0 + e, hang);
                const int p2 = a.relpos[ro + e];
                const T prod = lv2 * u;
                x[p2] = x[p2] - prod;
            }
            if (kLds) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            l0 = l0n;
            nl = nln;
            ro = ron;
            lv = lvn;
            pos = posn;
            l0n = l0nn;
            nln = nlnn;
            ron = ronn;
            lvn = lvnn;
            posn = posnn;
        }
        rp += __shfl(off_l + nl_l, cnt - 1, 64);
    }
}

// The update chain of column j from the flat update list [rp, re) (column staged in LDS at x):
// a round loads 64 updates at once, lane t holding update rp + t (the F index of its L entry,
// its target position and the position of its source's U entry), and their L values; then
// the sources of the round are applied one after another in ascending step (the updates of
// one source are consecutive in the list and go to distinct positions, so its lanes apply
// them together), each update as x[pos] = x[pos] - L * x[slot] from LDS.  The next round's
// metadata is in flight while a round is applied.
static_assert(kRefactorLds <= 65535, "update-list slots of LDS-staged columns fit 16 bits");

template <typename T, bool kLds>
__device__ void refactor_flat(const RefactorArgs<T> &a, int64_t rp, int64_t re, T *x) {
    const int lane = threadIdx.x & 63;
    unsigned int *hang = &a.ctl->hang;
    int src = 0, pos = 0, slot = 0;
    if (rp + lane < re) {
        src = a.relsrc[rp + lane];
        pos = a.relpos[rp + lane];
        slot = a.relslot[rp + lane];
    }
    for (int64_t b = rp; b < re; b += 64) {
        const int cnt = re - b < 64 ? (int)(re - b) : 64;
        const bool mine = lane < cnt;
        T lv = mine ? a.Ld[src] : T(0);
        const int cpos = pos, cslot = slot, csrc = src;
        // the next round's metadata
        src = pos = slot = 0;
        if (b + 64 + lane < re) {
            src = a.relsrc[b + 64 + lane];
            pos = a.relpos[b + 64 + lane];
            slot = a.relslot[b + 64 + lane];
        }
        const int prev = __shfl_up(cslot, 1, 64);
        unsigned long long starts = __ballot(mine && (lane == 0 || cslot != prev));
        while (starts) {
            const int g = __builtin_ctzll(starts);
            starts &= starts - 1;
            const int ge = starts ? __builtin_ctzll(starts) : cnt;
            if (lane >= g && lane < ge) {
                if (is_sentinel(lv)) lv = load_ready<T, 1>(a.Ld + csrc, hang);
                const T u = x[cslot];
                const T prod = lv * u;
                x[cpos] = x[cpos] - prod;
            }
            if (kLds) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            else __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Small columns of one dependency level, run side by side: group g of kGroupLanes lanes takes
// column src0 + g (g < b <= kGroups) with at most kGroupLen entries, staged in its share of
// the wavefront's LDS.  Each column gets the operations of the one-column path in the same order
// (staging and column max, updates in ascending source step, guard, division, publication),
// so the factors are the same bits.  Columns of one level never read each other's values, so
// no group waits for another group of its own wavefront.
constexpr int kGroupLanes = 16;
constexpr int kGroups = 64 / kGroupLanes;
constexpr int kGroupLen = 32;
static_assert(kGroupLen <= kRefactorLds / kGroups, "a group's column fits its LDS quarter");

template <typename T>
__device__ void refactor_group(const RefactorArgs<T> &a, T *xs_wave, int src0, int b, long long c0_l,
                               long long end_l, int nu_l, long long rp_l) {
    const int lane = threadIdx.x & 63, g = lane / kGroupLanes, gl = lane % kGroupLanes;
    const bool act = g < b;
    const int src = src0 + (act ? g : 0);
    const int64_t c0 = __shfl(c0_l, src, 64);
    const int64_t endc = __shfl(end_l, src, 64);
    const int nus = __shfl(nu_l, src, 64);
    int64_t rp = __shfl(rp_l, src, 64);
    const int len = act ? (int)(endc - c0) : 0;
    const int nu = act ? nus : 0;
    T *x = xs_wave + g * (kRefactorLds / kGroups);
    unsigned int *hang = &a.ctl->hang;
    T cm = 0;
    for (int e = gl; e < len; e += kGroupLanes) {
        const T v = a.F[c0 + e];
        x[e] = v;
        cm = fmax(cm, fabs(v));
    }
    for (int o = kGroupLanes / 2; o > 0; o >>= 1) cm = fmax(cm, __shfl_xor(cm, o, kGroupLanes));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int t0 = 0; t0 < nu; t0 += kGroupLanes) {
        const int cnt = nu - t0 < kGroupLanes ? nu - t0 : kGroupLanes;
        int64_t l0_l = 0;
        int nl_l = 0;
        if (gl < cnt) {
            const int k = a.fi[c0 + t0 + gl];
            l0_l = a.fp[k] + a.fdiag[k] + 1;
            nl_l = (int)(a.fp[k + 1] - l0_l);
        }
        int off_l = nl_l;
        for (int o = 1; o < kGroupLanes; o <<= 1) {
            const int v = __shfl_up(off_l, o, kGroupLanes);
            if (gl >= o) off_l += v;
        }
        off_l -= nl_l;
        for (int st = 0; st < cnt; ++st) {
            const int64_t l0 = __shfl(l0_l, st, kGroupLanes);
            const int nl = __shfl(nl_l, st, kGroupLanes);
            const int64_t ro = rp + __shfl(off_l, st, kGroupLanes);
            const T u = x[t0 + st];
            for (int e = gl; e < nl; e += kGroupLanes) {
                T lv = a.Ld[l0 + e];
                if (is_sentinel(lv)) lv = load_ready(a.Ld + l0 + e, hang);
                const int p2 = a.relpos[ro + e];
                const T prod = lv * u;
                x[p2] = x[p2] - prod;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        rp += __shfl(off_l + nl_l, cnt - 1, kGroupLanes);
    }
    if (!act) return;
    T d = x[nu];
    const T ur = unit_roundoff<T>();
    const T cmx = cm > T(0) ? cm : T(1);
    if (!(fabs(d) > ur * cmx) || !isfinite(d)) {
        d = (d < T(0) ? T(-1) : T(1)) * ur * cmx;
        if (gl == 0) {
            atomicAdd(&a.ctl->nguard, 1ull);
            if (a.guard_fail_policy) atomicOr(&a.ctl->guard_fail, 1u);
        }
    }
    for (int e = nu + 1 + gl; e < len; e += kGroupLanes) store_ready(a.Ld + c0 + e, x[e] / d);
    for (int e = gl; e < len; e += kGroupLanes) {
        T v = x[e];
        if (e == nu) v = d;
        else if (e > nu) v = v / d;
        a.Tv[a.f2t[c0 + e]] = v;
    }
}

// One column per lane: the columns of a lane item (one dependency level, at most kLaneLen
// entries each) run side by side, lane l taking col_order position cbeg + l.  Each column gets
// the operations of the one-column path in the same order (staging and column max, its
// updates in ascending source step from the flat update list, guard, division, publication),
// so the factors are the same bits.  Entry e of lane l's column sits at xs[e * 64 + l]; no
// lane reads another lane's entries, and columns of one level never wait for each other.
// A wavefront applies its columns' updates eight at a time: the eight metadata loads, then
// the eight L values, are in flight together.
template <typename T>
__device__ void refactor_lanes(const RefactorArgs<T> &a, T *xs, int64_t cbeg, int64_t cend) {
    const int lane = threadIdx.x & 63;
    const bool act = cbeg + lane < cend;
    int64_t c0 = 0, rp = 0, re = 0;
    int len = 0, nu = 0;
    if (act) {
        // the item's columns and update lists are side by side (col_order layout)
        const int64_t p = cbeg + lane;
        c0 = a.pc[p];
        len = (int)(a.pc[p + 1] - c0);
        nu = a.pnu[p];
        rp = a.pu[p];
        re = a.pu[p + 1];
    }
    T *x = xs + lane;
    T cm = 0;
#pragma unroll
    for (int h = 0; h < kLaneLen; h += 8) {
        T v[8];
        int sx[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) sx[e] = h + e < len ? a.fsrc[c0 + h + e] : -1;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = sx[e] >= 0 ? (T)a.kval[sx[e]] : T(0);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            x[(h + e) * 64] = v[e];
            cm = fmax(cm, fabs(v[e]));
        }
    }
    unsigned int *hang = &a.ctl->hang;
    for (int64_t b = rp; b < re; b += 8) {
        const int cnt = re - b < 8 ? (int)(re - b) : 8;
        int src[8], pos[8], slot[8];
        T lv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            src[t] = 0;
            pos[t] = 0;
            slot[t] = 0;
            if (t < cnt) {
                src[t] = a.relsrc[b + t];
                pos[t] = a.relpos[b + t];
                slot[t] = a.relslot[b + t];
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) lv[t] = t < cnt ? a.Ld[src[t]] : T(0);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t < cnt) {
                T l = lv[t];
                if (is_sentinel(l)) l = load_ready<T, 1>(a.Ld + src[t], hang);
                const T u = x[slot[t] * 64];
                const T prod = l * u;
                x[pos[t] * 64] = x[pos[t] * 64] - prod;
            }
        }
    }
    if (!act) return;
    T d = x[nu * 64];
    const T ur = unit_roundoff<T>();
    const T cmx = cm > T(0) ? cm : T(1);
    if (!(fabs(d) > ur * cmx) || !isfinite(d)) {
        d = (d < T(0) ? T(-1) : T(1)) * ur * cmx;
        atomicAdd(&a.ctl->nguard, 1ull);
        if (a.guard_fail_policy) atomicOr(&a.ctl->guard_fail, 1u);
    }
    // publish L(:,j) first (later columns wait for it), then the solve layout's copy
#pragma unroll
    for (int e = 1; e < kLaneLen; ++e)
        if (e > nu && e < len) store_ready(a.Ld + c0 + e, x[e * 64] / d);
#pragma unroll
    for (int e = 0; e < kLaneLen; ++e) {
        if (e < len) {
            T v = x[e * 64];
            if (e == nu) v = d;
            else if (e > nu) v = v / d;
            a.Tv[a.f2t[c0 + e]] = v;
        }
    }
}

// Several systems of one pattern refactored by one launch: slot b's value arrays and control
// block; the structure arrays are shared (every slot is bound to the same analysis).
template <typename T> struct RefactorBatch {
    int nslots;
    struct {
        T *F, *Tv, *Ld;
        Control *ctl;
        const double *kval;
    } slot[kMaxBatch];
};

// kFlat: the analysis built the flat update list (every factor of fewer than 2^31 entries);
// its columns run as lane items, from the flat list in LDS, or (longer than the LDS stage)
// from HBM.  Without it: lane groups, the per-source chain in LDS, or from HBM.  The two
// variants are separate kernels so that each is register-allocated for its own paths.
template <typename T, bool kFlat>
__global__ void __launch_bounds__(kCoopBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_refactor(RefactorArgs<T> args, RefactorBatch<T> batch) {
    __shared__ T lds[(kCoopBlock / 64) * kRefactorLds];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T *xs = lds + wid * kRefactorLds;
    (void)wid;
    // Columns are handed out in dependency-level order to running wavefronts only: the
    // earliest unfinished column is always held by a running wave whose earlier work is
    // done, so the kernel finishes whatever the residency.  The items (built by the analysis)
    // are lane items (up to 64 short columns of one level, one per lane), chunks of longer
    // columns of a wide level, and single columns of the narrow levels, so that no column of
    // a dependency chain waits behind another one grabbed by the same wave.
    // Items go round robin to kWorkQueues counters, item t to queue t % kWorkQueues (one counter
    // serializes its atomics: about 85 grabs per microsecond measured at 2M unknowns, which
    // bounded the hand-out).  Each queue is in level order, so the minimal unfinished item is
    // either held by a running wave or will be taken by one as long as every queue has a
    // resident block: block b serves queue b % kWorkQueues (blocks are dispatched in index
    // order, so any 8 resident blocks cover every queue), and a block whose queue is exhausted
    // moves on to the next queue.
    // With a batch of slots, hand-out position g is item g / nslots of slot g % nslots: the
    // slots' items interleave in level order, taken from the first slot's counters.
    unsigned int queue = blockIdx.x % kWorkQueues;
    int exhausted = 0;
    const int nslots = batch.nslots;
    for (;;) {
        const unsigned int g = queue + kWorkQueues * grab(&args.ctl->work_refactor[queue * 64], 1u);
        if ((int64_t)g >= args.nitems * nslots) {
            if (++exhausted == kWorkQueues) break;
            queue = (queue + 1) % kWorkQueues;
            continue;
        }
        const unsigned int it = nslots > 1 ? g / nslots : g;
        RefactorArgs<T> a = args;
        if (nslots > 1) {
            // selected by uniform compares, not by a dynamic index into the argument array
            // (which the compiler would copy to per-lane scratch memory)
            const int sb = (int)(g - it * nslots);
#pragma unroll
            for (int q = 1; q < kMaxBatch; ++q)
                if (q == sb) {
                    a.F = batch.slot[q].F;
                    a.Tv = batch.slot[q].Tv;
                    a.Ld = batch.slot[q].Ld;
                    a.ctl = batch.slot[q].ctl;
                    a.kval = batch.slot[q].kval;
                }
        }
        const int64_t cbeg = a.item[it], cend = a.item[it + 1];
        if (kFlat && a.item_lane[it]) {
            refactor_lanes<T>(a, xs, cbeg, cend);
            continue;
        }
        // metadata of the whole grab at once, lane l holding column cbeg + l (a grab has at
        // most 16 columns): one dependent round trip per grab instead of two per column
        int nu_l = 0, lev_l = -1;
        long long c0_l = 0, end_l = 0, rp_l = 0, rpe_l = 0;
        if (lane < cend - cbeg && kFlat) {
            const int64_t p = cbeg + lane;
            c0_l = a.pc[p];
            end_l = a.pc[p + 1];
            nu_l = a.pnu[p];
            rp_l = a.pu[p];
            rpe_l = a.pu[p + 1];
        } else if (lane < cend - cbeg) {
            const int j_l = a.order[cbeg + lane];
            lev_l = a.clev[cbeg + lane];
            c0_l = a.fp[j_l];
            end_l = a.fp[j_l + 1];
            nu_l = a.fdiag[j_l];
            rp_l = a.relptr[j_l];
            rpe_l = a.relptr[j_l + 1];
        }
        for (int64_t t = cbeg; t < cend;) {
        const int src = (int)(t - cbeg);
        if (!kFlat) {
            // a run of small columns of one level goes to lane groups, kGroups at a time
            const int lev0 = __shfl(lev_l, src, 64);
            int b = 0;
            while (b < kGroups && t + b < cend) {
                const int sb = src + b;
                const int lenb = (int)(__shfl(end_l, sb, 64) - __shfl(c0_l, sb, 64));
                if (__shfl(lev_l, sb, 64) != lev0 || lenb > kGroupLen) break;
                ++b;
            }
            if (b >= 2) {
                refactor_group<T>(a, xs, src, b, c0_l, end_l, nu_l, rp_l);
                t += b;
                continue;
            }
        }
        ++t;
        const int64_t c0 = __shfl(c0_l, src, 64);
        const int len = (int)(__shfl(end_l, src, 64) - c0);
        const int nu = __shfl(nu_l, src, 64);
        const int64_t rpj = __shfl(rp_l, src, 64);
        const bool in_lds = len <= kRefactorLds;
        T cm = 0;
        for (int e = lane; e < len; e += 64) {
            T v;
            if (kFlat) {
                // the column's values come straight from K (F is not initialized by the ingest)
                const int sx = a.fsrc[c0 + e];
                v = sx >= 0 ? (T)a.kval[sx] : T(0);
                if (!in_lds) a.F[c0 + e] = v;
            } else {
                v = a.F[c0 + e];
            }
            if (in_lds) xs[e] = v;
            cm = fmax(cm, fabs(v));
        }
        cm = wave_max(cm);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (kFlat && in_lds) refactor_flat<T, true>(a, rpj, __shfl(rpe_l, src, 64), xs);
        else if (kFlat) refactor_flat<T, false>(a, rpj, __shfl(rpe_l, src, 64), a.F + c0);
        else if (in_lds) refactor_chain<T, true>(a, rpj, c0, nu, xs);
        else refactor_chain<T, false>(a, rpj, c0, nu, a.F + c0);
        const T *x = in_lds ? xs : a.F + c0;
        T d = x[nu];
        const T ur = unit_roundoff<T>();
        const T cmx = cm > T(0) ? cm : T(1);
        if (!(fabs(d) > ur * cmx) || !isfinite(d)) {
            d = (d < T(0) ? T(-1) : T(1)) * ur * cmx;
            if (lane == 0) {
                atomicAdd(&a.ctl->nguard, 1ull);
                if (a.guard_fail_policy) atomicOr(&a.ctl->guard_fail, 1u);
            }
        }
        // publish L(:,j) first (entry by entry; later columns wait for it), then the copy in
        // the solve layout (whose scatter index is a load of its own).  F is only the working
        // column of the paths that update in HBM: nothing reads its final values, and the
        // host reads the factors back from the solve layout (without the F copy the 2M
        // refactorization takes 1.05 instead of 1.11 ms)
        for (int e = nu + 1 + lane; e < len; e += 64) store_ready(a.Ld + c0 + e, x[e] / d);
        for (int e = lane; e < len; e += 64) {
            T v = x[e];
            if (e == nu) v = d;
            else if (e > nu) v = v / d;
            a.Tv[a.f2t[c0 + e]] = v;
        }
        }
    }
}

// ---------------------------------------------------------------------------------------
// triangular solves in solve layout (step space), by tiles of segments
// ---------------------------------------------------------------------------------------

template <typename T> struct TrsvArgs {
    int64_t ntiles;
    const int32_t *seg_row;   // segment start in rows
    const int32_t *seg_lg;    // log2 lanes per row of each segment
    const int32_t *rows;      // solve order
    const int64_t *row_ent;   // first packed entry of each position of rows
    const int32_t *ent_ref;   // LDS slot (staged tile) or source row (unstaged tile)
    const int32_t *ext_src;   // source row of each external
    const int32_t *seg_dofs;  // dense segment: its block's offset in the tile's dense values
    const T *val;             // packed entry values, then dense blocks
    const T *diag;            // upper only: diagonal of U in step order
    const int32_t *tdesc;     // per tile, kTileDesc ints: its segments, rows, entries, externals,
                              // dense values and staged flag (one scalar load per tile)
    const double *rhs64;      // lower: right-hand side (gathered by rsrc)
    const int32_t *rsrc;      // lower: per position of rows, the right-hand-side entry it reads
    const T *rhs_step;        // upper: L-solve result (step order)
    T *out;                   // step-order result; sentinel on entry
    double *xout;             // upper: solution, scattered by qpos
    const int32_t *qpos;      // upper: per position of rows, the solution entry it writes
    const Control *stopflag;  // when non-null, skip if the FGMRES cycle has stopped
    unsigned int *work;       // tile counter (zeroed before the launch)
    unsigned int *hang;
};

// A lane's share of a row from LDS: acc + vals[e] * xs[refs[e]] for e = e0, e0 + g, ... < e1,
// added in that order; four entries at a time, their references, values and operands loaded
// together (two dependent LDS rounds per four entries).
template <typename T>
__device__ __forceinline__ T lane_row_sum(T acc, int e0, int e1, int g, const T *vals, const uint16_t *refs,
                                          const T *xs) {
    for (int e = e0; e < e1; e += 4 * g) {
        int c[4];
        T v[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int eu = e + u * g;
            c[u] = eu < e1 ? refs[eu] : 0;
            v[u] = eu < e1 ? vals[eu] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = e + u * g < e1 ? xs[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e + u * g < e1) {
                const T prod = v[u] * x[u];
                acc = acc + prod;
            }
    }
    return acc;
}

// Per tile descriptor: s0, s1, rb, re, eb (lo, hi), ne, xb, nx, db (lo, hi), nd, staged.
constexpr int kTileDesc = 16;
// Staging loads per thread and pass (a pass covers 2,048 entries, 512 rows, 512 externals and
// 1,024 dense values).
constexpr int kStageEnt = 8, kStageRow = 2, kStageExt = 2, kStageDense = 4;

// Triangular solve by tiles.  Tiles are handed out in order to running blocks; a tile's
// references point to earlier tiles or to earlier segments of the same tile, so the earliest
// unfinished tile is always held by a running block that can finish it.
//
// A staged tile is first copied into LDS with coalesced loads: its packed entries (values and
// 16-bit slot references), each row's id, entry offset and right-hand-side data, and the
// solution values of its externals (rows of earlier tiles; an entry still holding the
// sentinel is polled until its producer stores it).  The segments then run from LDS only,
// one pass of the block each (a lane group owns at most one row) with a barrier in between:
// no global load, hence no wait on memory, inside the segment loop; results go to LDS for
// the following segments and to the global solution with one coherent store each (every
// solution entry is its own ready flag).  An unstaged tile (one long row) is solved by one
// wavefront reading its entries and sources from global memory.
// Value of another lane selected by a DPP control (row shifts fill 0 past the row edge; rows
// outside kRowMask return 0), applied to each 32-bit half of a double.
template <int kCtrl, int kRowMask> __device__ __forceinline__ double dpp_get(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, kRowMask, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <int kCtrl, int kRowMask> __device__ __forceinline__ float dpp_get(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xF, true));
}

// Sum over aligned groups of 2^lg lanes (lg <= 6), complete in each group's last lane: an
// inclusive shift-add scan within rows of 16 lanes (row_shr 1, 2, 4, 8), then the row
// broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3.  Register-only.
template <typename T> __device__ __forceinline__ T group_sum_last(T v, int lg) {
    if (lg >= 1) v = v + dpp_get<0x111, 0xF>(v);
    if (lg >= 2) v = v + dpp_get<0x112, 0xF>(v);
    if (lg >= 3) v = v + dpp_get<0x114, 0xF>(v);
    if (lg >= 4) v = v + dpp_get<0x118, 0xF>(v);
    if (lg >= 5) v = v + dpp_get<0x142, 0xA>(v);
    if (lg >= 6) v = v + dpp_get<0x143, 0xC>(v);
    return v;
}

// Value of lane l (uniform) of v.
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Read-only schedule data seen through the constant address space: with a uniform index the
// compiler loads it through the scalar cache, so waiting for it never waits for the
// kernel's outstanding vector stores.
template <typename P> __device__ __forceinline__ const __attribute__((address_space(4))) P *uniform_ro(const P *p) {
    return (const __attribute__((address_space(4))) P *)p;
}

template <typename T, bool kLower, bool kDense>
__global__ void __launch_bounds__(kTileThreads) k_trsv(TrsvArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];  // the tile budget, sized at launch
    __shared__ T ys[kDenseRows];  // dense segment: rows' right-hand sides minus earlier terms
    __shared__ unsigned int tile_sh;
    if (a.stopflag && a.stopflag->stop) return;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) tile_sh = atomicAdd(a.work, 1u);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane((int)tile_sh);
        __syncthreads();
        if ((int64_t)t >= a.ntiles) break;
        const auto seg_row = uniform_ro(a.seg_row);
        const auto seg_lg = uniform_ro(a.seg_lg);
        const auto td = uniform_ro(a.tdesc) + (int64_t)kTileDesc * t;
        const int s0 = td[0], s1 = td[1], rb = td[2], re = td[3];
        const int nr = re - rb;
        const int64_t eb = (int64_t)(((uint64_t)(uint32_t)td[5] << 32) | (uint32_t)td[4]);
        const int ne = td[6];
        if (!td[12]) {
            // one row, one wavefront, entries and sources in global memory
            if (tid < 64) {
                const int i = a.rows[rb];
                T acc = 0;
                for (int e = tid; e < ne; e += 64) {
                    const int c = a.ent_ref[eb + e];
                    T xk = a.out[c];
                    if (is_sentinel(xk)) xk = load_ready<T, 1>(a.out + c, a.hang);
                    const T prod = a.val[eb + e] * xk;
                    acc = acc + prod;
                }
                for (int o = 1; o < 64; o <<= 1) acc = acc + __shfl_xor(acc, o, 64);
                if (tid == 0) {
                    T res;
                    if (kLower) res = (T)a.rhs64[a.rsrc[rb]] - acc;
                    else res = (a.rhs_step[i] - acc) / a.diag[i];
                    store_ready(a.out + i, res);
                    if (!kLower) a.xout[a.qpos[rb]] = (double)res;
                }
            }
            __syncthreads();
            continue;
        }
        const int xb = td[7], nx = td[8];
        const int64_t db = (int64_t)(((uint64_t)(uint32_t)td[10] << 32) | (uint32_t)td[9]);
        const int nd = td[11];
        const auto seg_dofs = uniform_ro(a.seg_dofs);
        // LDS carve-up: 8-byte arrays first, then 4-byte, then 2-byte
        T *xs = reinterpret_cast<T *>(smem);       // nr + nx solution slots
        T *rhs = xs + nr + nx;                     // nr
        T *dg = rhs + nr;                          // nr (upper)
        T *vals = dg + nr;                         // ne
        T *dvs = vals + ne;                        // nd: dense blocks
        int32_t *rid = reinterpret_cast<int32_t *>(dvs + nd);  // nr
        int32_t *qid = rid + nr;                   // nr (upper)
        int32_t *roff = qid + nr;                  // nr + 1
        uint16_t *refs = reinterpret_cast<uint16_t *>(roff + nr + 1);  // ne
        // Staging in passes: a pass issues every first-level load it covers (kStageEnt entries,
        // kStageRow rows, kStageExt externals and kStageDense dense values per thread), then the
        // dependent ones (right-hand sides, diagonals, externals' values), then writes LDS, so a
        // tile of the usual size is staged in two rounds of memory latency.
        for (int pe = 0, pr = 0, px = 0, pd = 0; pe < ne || pr < nr || px < nx || pd < nd;
             pe += kStageEnt * kTileThreads, pr += kStageRow * kTileThreads, px += kStageExt * kTileThreads,
             pd += kStageDense * kTileThreads) {
            T v[kStageEnt], dv[kStageDense], rv[kStageRow], gv[kStageRow], xv[kStageExt];
            int c[kStageEnt], ri[kStageRow], rs[kStageRow], xc[kStageExt];
            int64_t ro[kStageRow];
#pragma unroll
            for (int u = 0; u < kStageEnt; ++u) {
                const int k = pe + tid + u * kTileThreads;
                v[u] = k < ne ? a.val[eb + k] : T(0);
                c[u] = k < ne ? a.ent_ref[eb + k] : 0;
            }
#pragma unroll
            for (int u = 0; u < kStageDense; ++u) {
                const int k = pd + tid + u * kTileThreads;
                dv[u] = k < nd ? a.val[db + k] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kStageRow; ++u) {
                const int r = pr + tid + u * kTileThreads;
                ri[u] = r < nr ? a.rows[rb + r] : 0;
                ro[u] = r < nr ? a.row_ent[rb + r] : eb;
                rs[u] = r < nr ? (kLower ? a.rsrc[rb + r] : a.qpos[rb + r]) : 0;
            }
#pragma unroll
            for (int u = 0; u < kStageExt; ++u) {
                const int k = px + tid + u * kTileThreads;
                xc[u] = k < nx ? a.ext_src[xb + k] : 0;
            }
            // dependent loads
#pragma unroll
            for (int u = 0; u < kStageRow; ++u) {
                const int r = pr + tid + u * kTileThreads;
                rv[u] = T(0);
                gv[u] = T(1);
                if (r < nr) {
                    if (kLower) {
                        rv[u] = (T)a.rhs64[rs[u]];
                    } else {
                        rv[u] = a.rhs_step[ri[u]];
                        gv[u] = a.diag[ri[u]];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kStageExt; ++u) {
                const int k = px + tid + u * kTileThreads;
                xv[u] = k < nx ? a.out[xc[u]] : T(0);
            }
            // LDS
#pragma unroll
            for (int u = 0; u < kStageEnt; ++u) {
                const int k = pe + tid + u * kTileThreads;
                if (k < ne) {
                    vals[k] = v[u];
                    refs[k] = (uint16_t)c[u];
                }
            }
#pragma unroll
            for (int u = 0; u < kStageDense; ++u) {
                const int k = pd + tid + u * kTileThreads;
                if (k < nd) dvs[k] = dv[u];
            }
#pragma unroll
            for (int u = 0; u < kStageRow; ++u) {
                const int r = pr + tid + u * kTileThreads;
                if (r < nr) {
                    rid[r] = ri[u];
                    roff[r] = (int32_t)(ro[u] - eb);
                    rhs[r] = rv[u];
                    if (!kLower) {
                        dg[r] = T(1) / gv[u];  // reciprocal: one multiply per row in the segments
                        qid[r] = rs[u];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kStageExt; ++u) {
                const int k = px + tid + u * kTileThreads;
                if (k < nx) {
                    T x = xv[u];
                    if (is_sentinel(x)) x = load_ready<T, 1>(a.out + xc[u], a.hang);
                    xs[nr + k] = x;
                }
            }
        }
        if (tid == 0) roff[nr] = ne;
        __syncthreads();
        // A wavefront segment is solved by wavefront 0 alone: between two such segments no
        // block barrier is needed (a wavefront's LDS accesses complete in order).
        bool prev_wave = false;
        for (int sg = s0; sg < s1; ++sg) {
            const int lb = seg_row[sg] - rb, le = seg_row[sg + 1] - rb;
            const int code = seg_lg[sg];
            const bool wave = (code & kSegWave) != 0;
            const int lg = code & 0xF;
            const int g = 1 << lg;
            if (sg > s0 && !(wave && prev_wave)) __syncthreads();
            if (kDense && (code & kSegDense)) {
                // phase A (block pass): each row's terms from earlier segments and tiles
                const int r = lb + (tid >> lg);
                T acc = 0;
                if (r < le) {
                    const int e1 = roff[r + 1];
                    for (int e = roff[r] + (tid & (g - 1)); e < e1; e += g) {
                        const T prod = vals[e] * xs[refs[e]];
                        acc = acc + prod;
                    }
                }
                acc = group_sum_last(acc, lg);
                if (r < le && (tid & (g - 1)) == g - 1) ys[r - lb] = rhs[r] - acc;
                __syncthreads();
                // phase B (wavefront 0): column sweep over the dense strictly lower block,
                // lane l owns row l; x_c is broadcast from lane c once its row is final
                if (tid < 64) {
                    const int m = le - lb, l = tid;
                    const T *D = dvs + seg_dofs[sg];
                    T y = l < m ? ys[l] : T(0);
                    const T inv = (!kLower && l < m) ? dg[lb + l] : T(1);
                    // lane l's coefficient of column c (0 above the diagonal), read four
                    // columns ahead of its use
                    auto coef = [&](int c) -> T {
                        return (l > c && l < m) ? D[c * m - c * (c + 1) / 2 + (l - c - 1)] : T(0);
                    };
                    T q0 = coef(0), q1 = coef(1), q2 = coef(2), q3 = coef(3);
                    for (int c = 0; c < m; c += 4) {
                        const T n0 = coef(c + 4), n1 = coef(c + 5), n2 = coef(c + 6), n3 = coef(c + 7);
                        const T qs[4] = {q0, q1, q2, q3};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (c + u < m) {
                                const T xc = lane_value(kLower ? y : y * inv, c + u);
                                if (l > c + u) {
                                    const T prod = qs[u] * xc;
                                    y = y - prod;
                                }
                            }
                        }
                        q0 = n0;
                        q1 = n1;
                        q2 = n2;
                        q3 = n3;
                    }
                    if (l < m) {
                        const T res = kLower ? y : y * inv;
                        const int r2 = lb + l;
                        xs[r2] = res;
                        store_ready(a.out + rid[r2], res);
                        if (!kLower) a.xout[qid[r2]] = (double)res;
                    }
                }
                prev_wave = true;  // the last writer is wavefront 0
                continue;
            }
            prev_wave = wave;
            if (wave && tid >= 64) continue;
            const int r = lb + (tid >> lg);
            T acc = 0;
            if (r < le) {
                const int e1 = roff[r + 1];
                int e = roff[r] + (tid & (g - 1));
                for (; e + 3 * g < e1; e += 4 * g) {  // operands of four entries in flight
                    const int c0 = refs[e], c1 = refs[e + g], c2 = refs[e + 2 * g], c3 = refs[e + 3 * g];
                    const T v0 = vals[e], v1 = vals[e + g], v2 = vals[e + 2 * g], v3 = vals[e + 3 * g];
                    const T p0 = v0 * xs[c0], p1 = v1 * xs[c1], p2 = v2 * xs[c2], p3 = v3 * xs[c3];
                    acc = acc + p0;
                    acc = acc + p1;
                    acc = acc + p2;
                    acc = acc + p3;
                }
                for (; e < e1; e += g) {
                    const T prod = vals[e] * xs[refs[e]];
                    acc = acc + prod;
                }
            }
            acc = group_sum_last(acc, lg);
            if (r < le && (tid & (g - 1)) == g - 1) {
                T res;
                if (kLower) res = rhs[r] - acc;
                else res = (rhs[r] - acc) * dg[r];
                xs[r] = res;
                store_ready(a.out + rid[r], res);
                if (!kLower) a.xout[qid[r]] = (double)res;
            }
        }
        __syncthreads();
    }
}

// Arms the two solve vectors with the sentinel and zeroes the tile counters of the two
// sweeps (and the wait-failure flag, when given).
template <typename T>
__global__ void k_fill_sentinel(int64_t n, T *a, T *b, unsigned int *work_lower, unsigned int *work_upper,
                                unsigned int *hang) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *work_lower = 0;
        *work_upper = 0;
        if (hang) *hang = 0;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        a[i] = sentinel<T>();
        b[i] = sentinel<T>();
    }
}

// ---------------------------------------------------------------------------------------
// Krylov kernels (FP64).  Streaming grid: G <= kStreamGridMax blocks of kStreamBlock threads,
// block b owns a contiguous chunk of rows and writes its partial sums to
// part[b * kPartStride + t] with plain stores; the NEXT kernel reduces the partials in every
// block, in block order (deterministic, identical in every block), so no reduction needs a
// memory fence: the kernel boundary makes the partials visible.  Three partial buffers
// rotate so a kernel never overwrites the partials it is reading.
// ---------------------------------------------------------------------------------------

constexpr int kPartStride = 2 * kRestartMax + 4;  // room for the 2 (j + 1) dots of a DCGS2 step

struct KrylovArgs {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    const double *kval;
    double *V;        // (R+1) columns of n
    double *Z;        // R columns of n
    double *w;
    double *part;     // 3 buffers of kStreamGridMax * kPartStride
    Control *ctl;
};

__device__ __forceinline__ double *partbuf(const KrylovArgs &a, int which) {
    return a.part + (int64_t)which * kStreamGridMax * kPartStride;
}

// Sum of partial column t over the G blocks of the previous kernel (fixed order; one thread).
__device__ __forceinline__ double reduce_part(const double *buf, int G, int t) {
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += buf[(int64_t)b * kPartStride + t];
    return s;
}

// Per-column partial sums of one block without a barrier per column: each wavefront reduces
// its value with shuffles and lane 0 parks it in red[t][wave]; block_cols_finish() (one
// barrier) then adds the kStreamBlock/64 wave values of column t in wave order.
__device__ __forceinline__ void block_col_put(double v, int t, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[t * (kStreamBlock / 64) + (threadIdx.x >> 6)] = v;
}
__device__ __forceinline__ double block_col_get(const double *red, int t) {
    double s = 0.0;
    for (int w = 0; w < kStreamBlock / 64; ++w) s += red[t * (kStreamBlock / 64) + w];
    return s;
}

// Reduces columns 0..m-1 of buf (G <= kStreamGridMax block rows) into out[] (shared): thread
// b adds rows b, b + kStreamBlock, ... in that order, then per-column sums in a fixed tree
// (identical in every block).
__device__ void reduce_cols(const double *buf, int G, int m, double *out, double *red) {
    const int b = threadIdx.x;
    for (int t = 0; t < m; ++t) {
        double v = 0.0;
        for (int r = b; r < G; r += kStreamBlock) v += buf[(int64_t)r * kPartStride + t];
        block_col_put(v, t, red);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += blockDim.x) out[t] = block_col_get(red, t);
    __syncthreads();
}

// w = K z_j; partials (buffer 0): V_t . w for t <= j, and w . w at t = j + 1
__global__ void __launch_bounds__(kStreamBlock) k_spmv_dots(KrylovArgs a, int j) {
    __shared__ double red[(kRestartMax + 2) * (kStreamBlock / 64)];
    if (a.ctl->stop) return;  // enqueued ahead of the host's stop test
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    const double *z = a.Z + (int64_t)j * a.n;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) a.w[i] = row_dot(a.rp, a.ci, a.kval, z, i);
    __syncthreads();
    double *out = partbuf(a, 0) + (int64_t)blockIdx.x * kPartStride;
    for (int t = 0; t <= j + 1; ++t) {
        const double *v = t <= j ? a.V + (int64_t)t * a.n : a.w;
        double s = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += v[i] * a.w[i];
        block_col_put(s, t, red);
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j + 1; t += blockDim.x) out[t] = block_col_get(red, t);
}

// h1 = reduce(buffer 0); w -= V h1; partials (buffer 1): V_t . w (second CGS pass)
__global__ void __launch_bounds__(kStreamBlock) k_cgs_pass2(KrylovArgs a, int j) {
    __shared__ double red[(kRestartMax + 2) * (kStreamBlock / 64)];
    __shared__ double h[kRestartMax + 2];
    if (a.ctl->stop) return;
    const int G = gridDim.x;
    reduce_cols(partbuf(a, 0), G, j + 2, h, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int t = 0; t <= j; ++t) a.ctl->h1[t] = h[t];
        a.ctl->wnorm_in = sqrt(h[j + 1]);
    }
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double s = a.w[i];
        for (int t = 0; t <= j; ++t) {
            const double prod = a.V[(int64_t)t * a.n + i] * h[t];
            s = s - prod;
        }
        a.w[i] = s;
    }
    __syncthreads();
    double *out = partbuf(a, 1) + (int64_t)blockIdx.x * kPartStride;
    for (int t = 0; t <= j; ++t) {
        const double *v = a.V + (int64_t)t * a.n;
        double s = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += v[i] * a.w[i];
        block_col_put(s, t, red);
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j; t += blockDim.x) out[t] = block_col_get(red, t);
}

// h2 = reduce(buffer 1); w -= V h2; partial (buffer 2): w . w
__global__ void __launch_bounds__(kStreamBlock) k_cgs_finish(KrylovArgs a, int j) {
    __shared__ double red[(kRestartMax + 2) * (kStreamBlock / 64)];
    __shared__ double h[kRestartMax + 1];
    if (a.ctl->stop) return;
    const int G = gridDim.x;
    reduce_cols(partbuf(a, 1), G, j + 1, h, red);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int t = 0; t <= j; ++t) a.ctl->h2[t] = h[t];
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    double ss = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double s = a.w[i];
        for (int t = 0; t <= j; ++t) {
            const double prod = a.V[(int64_t)t * a.n + i] * h[t];
            s = s - prod;
        }
        a.w[i] = s;
        ss += s * s;
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) partbuf(a, 2)[(int64_t)blockIdx.x * kPartStride] = ss;
}

// Closes Arnoldi column j (thread 0 of every block, identical results): col[0..j] are the
// Gram-Schmidt coefficients, hn the new subdiagonal entry; applies the previous rotations
// and a new Givens rotation, forms the estimated residual |g_{j+1}| and the stop test.
// Block 0 stores the column, rotation, right-hand side and the host record r of the step.  Every
// value another block reads here (g[j], cs, sn, inner_tol) is left untouched in this launch.
// sh receives hn, breakdown, stop.
__device__ void arnoldi_close(Control *c, int j, int restart, double hn, double wnorm_in, double *col,
                              StepRecord *r, unsigned long long token, double *sh) {
    col[j + 1] = hn;
    for (int t = 0; t < j; ++t) {
        const double x0 = col[t], x1 = col[t + 1];
        col[t] = c->cs[t] * x0 + c->sn[t] * x1;
        col[t + 1] = -c->sn[t] * x0 + c->cs[t] * x1;
    }
    const double rr = hypot(col[j], col[j + 1]);
    double cs = 1.0, sn = 0.0;
    if (rr != 0.0) {
        cs = col[j] / rr;
        sn = col[j + 1] / rr;
    }
    col[j] = rr;
    const double gj = c->g[j];
    const double gj1 = -sn * gj;
    const double est = fabs(gj1);
    const int brk = !(hn > 1e-14 * wnorm_in);
    const int stop = est <= c->inner_tol || brk || j + 1 >= restart;
    sh[0] = hn;
    sh[1] = brk;
    sh[2] = stop;
    if (blockIdx.x == 0) {
        c->cs[j] = cs;
        c->sn[j] = sn;
        c->g[j + 1] = gj1;
        c->gr[j] = cs * gj;
        for (int t = 0; t <= j; ++t) c->H[j * (kRestartMax + 1) + t] = col[t];
        c->hn = hn;
        c->est = est;
        c->jdone = j + 1;
        c->breakdown = brk;
        c->stop = stop;
        if (!stop) {
            c->work_lower = 0;
            c->work_upper = 0;
        }
        __hip_atomic_store(&r->est, est, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->jdone, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->hang, c->hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->token, token, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// hn = ||w|| (reduce buffer 2); Hessenberg column h1 + h2, rotation and stop test
// (arnoldi_close); then v_{j+1} = w / hn unless the step broke down, and the solve
// sentinels are re-armed when the cycle goes on.
template <typename T>
__global__ void __launch_bounds__(kStreamBlock) k_normalize(KrylovArgs a, int j, int restart, T *s1, T *s2,
                                                            StepRecord *rec, unsigned long long token) {
    __shared__ double sh[3];
    __shared__ double red[kStreamBlock / 64];
    __shared__ double hsq[1];
    Control *c = a.ctl;
    if (c->stop) return;
    reduce_cols(partbuf(a, 2), gridDim.x, 1, hsq, red);
    if (threadIdx.x == 0) {
        double col[kRestartMax + 1];
        for (int t = 0; t <= j; ++t) col[t] = c->h1[t] + c->h2[t];
        arnoldi_close(c, j, restart, sqrt(hsq[0]), c->wnorm_in, col, rec + j, token, sh);
    }
    __syncthreads();
    const double hn = sh[0];
    const bool write_v = sh[1] == 0.0;
    const bool rearm = sh[2] == 0.0;
    double *v = a.V + (int64_t)(j + 1) * a.n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        if (write_v) v[i] = a.w[i] / hn;
        if (rearm) {
            s1[i] = sentinel<T>();
            s2[i] = sentinel<T>();
        }
    }
}

// Delayed CGS2 (Bielich et al., Parallel Computing 2022), one of the low-synchronization
// FGMRES variants of Section 2.1: one global reduction per Arnoldi step.  Step j works on u_j,
// the vector left by one Gram-Schmidt pass (V slot j; u_0 = v_0 is final).  Its second pass
// and normalization are deferred to step j and share the reduction with w = K M^-1 u_j:
//   s_t = v_t.u_j, c_t = v_t.w (t < j), alpha = u_j.u_j, d = u_j.w
//   beta = sqrt(alpha - |s|^2), v_j = (u_j - V s) / beta: column j - 1 becomes final,
//     (p + s, beta) with p its one-pass part, and is rotated and tested (arnoldi_close)
//   z_j = (M^-1 u_j - Z s) / beta = M^-1 v_j
//   K z_j = (w - V Hbar s) / beta by the Arnoldi relation K Z = V Hbar, so with
//     e = V^T w (e_t = c_t, e_j = (d - s.c) / beta) the next one-pass column is
//     p = (e - Hbar s) / beta and u_{j+1} = (w - V e) / beta.
// beta = 1 and s = () at j = 0; the closing step j = R only finishes column R - 1.
// The estimate of column j - 1 is thus known one preconditioner application later than
// with CGS2, so a cycle that converges spends one application more.

// w = K z_j (when matvec); partials (buffer 0): V_t . w at t and V_t . u_j at j + 1 + t, t <= j
__global__ void __launch_bounds__(kStreamBlock) k_dcgs2_dots(KrylovArgs a, int j, int matvec) {
    __shared__ double red[(2 * kRestartMax + 4) * (kStreamBlock / 64)];
    if (a.ctl->stop) return;
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    if (matvec) {
        const double *z = a.Z + (int64_t)j * a.n;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) a.w[i] = row_dot(a.rp, a.ci, a.kval, z, i);
    }
    __syncthreads();
    const double *u = a.V + (int64_t)j * a.n;
    for (int t = 0; t <= j; ++t) {
        const double *v = a.V + (int64_t)t * a.n;
        double sw = 0.0, su = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const double vi = v[i];
            if (matvec) sw += vi * a.w[i];
            su += vi * u[i];
        }
        block_col_put(sw, t, red);
        block_col_put(su, j + 1 + t, red);
    }
    __syncthreads();
    double *out = partbuf(a, 0) + (int64_t)blockIdx.x * kPartStride;
    for (int t = threadIdx.x; t < 2 * (j + 1); t += blockDim.x) out[t] = block_col_get(red, t);
}

// The rest of DCGS2 step j (see above): every block reduces the partials and forms the same
// scalars in thread 0; block 0 stores the final column j - 1 (before rotation, in Hbar; and
// rotated, in H), the one-pass column j (in hp[j & 1], read by the next step, so that no
// block reads what block 0 writes in this launch) and the step's host record.  Then
// v_j, z_j and u_{j+1} are formed in one pass over V and Z, and the solve sentinels re-armed.
template <typename T>
__global__ void __launch_bounds__(kStreamBlock) k_dcgs2(KrylovArgs a, int j, int restart, T *s1, T *s2,
                                                        StepRecord *rec, unsigned long long token) {
    __shared__ double red[(2 * kRestartMax + 4) * (kStreamBlock / 64)];
    __shared__ double cw[2 * kRestartMax + 2];  // c_t (t < j), d at j; s_t at j + 1 + t, alpha at 2j + 1
    __shared__ double sh[5];                    // hn, breakdown, stop (arnoldi_close); beta, e_j
    Control *c = a.ctl;
    if (c->stop) return;
    reduce_cols(partbuf(a, 0), gridDim.x, 2 * (j + 1), cw, red);
    if (threadIdx.x == 0) {
        const double *sv = cw + j + 1;
        double beta = 1.0;
        sh[2] = 0.0;
        double fin[kRestartMax + 2];  // final column j - 1 before rotation
        if (j > 0) {
            double ss = 0.0;
            for (int t = 0; t < j; ++t) ss += sv[t] * sv[t];
            const double d2 = sv[j] - ss;
            beta = d2 > 0.0 ? sqrt(d2) : 0.0;
            const double *p = c->hp[(j - 1) & 1];
            double cn = 0.0;
            for (int t = 0; t < j; ++t) fin[t] = p[t] + sv[t];
            fin[j] = beta;
            for (int t = 0; t <= j; ++t) cn += fin[t] * fin[t];
            double col[kRestartMax + 2];
            for (int t = 0; t <= j; ++t) col[t] = fin[t];
            if (blockIdx.x == 0)
                for (int t = 0; t <= j; ++t) c->Hbar[(j - 1) * (kRestartMax + 1) + t] = fin[t];
            arnoldi_close(c, j - 1, restart, beta, sqrt(cn), col, rec + j, token, sh);
        } else if (blockIdx.x == 0) {
            c->work_lower = 0;
            c->work_upper = 0;
            StepRecord *r = rec;
            __hip_atomic_store(&r->est, c->est, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&r->jdone, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&r->hang, c->hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&r->stop, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&r->token, token, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        sh[3] = beta;
        if (sh[2] == 0.0) {
            // one-pass column j: p = (e - Hbar s) / beta, Hbar's columns 0..j-2 from earlier
            // steps and column j - 1 from fin
            double sc = 0.0;
            for (int t = 0; t < j; ++t) sc += sv[t] * cw[t];
            const double ej = (cw[j] - sc) / beta;
            sh[4] = ej;
            if (blockIdx.x == 0) {
                double *pn = c->hp[j & 1];
                for (int t = 0; t <= j; ++t) {
                    double hs = 0.0;
                    for (int k = 0; k < j; ++k) {
                        const double hk = k == j - 1 ? fin[t] : (t <= k + 1 ? c->Hbar[k * (kRestartMax + 1) + t] : 0.0);
                        hs += hk * sv[k];
                    }
                    const double et = t < j ? cw[t] : ej;
                    pn[t] = (et - hs) / beta;
                }
            }
        }
    }
    __syncthreads();
    if (sh[2] != 0.0) return;  // the cycle ends: no further vector is needed
    const double beta = sh[3], ej = sh[4];
    const double *sv = cw + j + 1;
    double *vj = a.V + (int64_t)j * a.n;
    double *zj = a.Z + (int64_t)j * a.n;
    double *un = a.V + (int64_t)(j + 1) * a.n;
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double vs = 0.0, vc = 0.0, zs = 0.0;
        for (int t = 0; t < j; ++t) {
            const double vt = a.V[(int64_t)t * a.n + i];
            vs += vt * sv[t];
            vc += vt * cw[t];
            zs += a.Z[(int64_t)t * a.n + i] * sv[t];
        }
        double v = vj[i];
        if (j > 0) {
            v = (v - vs) / beta;
            vj[i] = v;
            zj[i] = (zj[i] - zs) / beta;
        }
        un[i] = (a.w[i] - vc - ej * v) / beta;
        s1[i] = sentinel<T>();
        s2[i] = sentinel<T>();
    }
}

// Row i of rho = b - K x in double-double: the pair (hi, lo) starts at (b_i, 0) and each
// product v*x enters as its exact pair (v*x rounded, and the rounding error from one fused
// multiply-add), added with the accurate double-word sum of Joldes, Muller and Popescu
// (ACM TOMS 2017, relative error <= 3u^2); the row is rounded once, to hi.
__device__ __forceinline__ void dd_accumulate(double &hi, double &lo, double v, double x) {
    const double ph = v * x;
    const double pl = fma(v, x, -ph);
    const double yh = -ph, yl = -pl;
    // exact sums of the high and of the low parts (Knuth)
    const double sh = hi + yh;
    const double sbv = sh - hi;
    const double sl = (hi - (sh - sbv)) + (yh - sbv);
    const double th = lo + yl;
    const double tbv = th - lo;
    const double tl = (lo - (th - tbv)) + (yl - tbv);
    // renormalize twice (Dekker: |sh| >= |c|, |vh| >= |w|)
    const double c = sl + th;
    const double vh = sh + c;
    const double vl = c - (vh - sh);
    const double w = tl + vl;
    const double zh = vh + w;
    lo = w - (zh - vh);
    hi = zh;
}

template <bool kDD>
__device__ __forceinline__ double resid_row(const KrylovArgs &a, const double *x, double bi, int64_t i) {
    if (kDD) {
        double hi = bi, lo = 0.0;
        const int64_t e = a.rp[i + 1];
        for (int64_t p = a.rp[i]; p < e; p += kRowBatch) {
            int c[kRowBatch];
            double v[kRowBatch], xv[kRowBatch];
#pragma unroll
            for (int t = 0; t < kRowBatch; ++t) {
                c[t] = p + t < e ? a.ci[p + t] : 0;
                v[t] = p + t < e ? a.kval[p + t] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < kRowBatch; ++t) xv[t] = p + t < e ? x[c[t]] : 0.0;
#pragma unroll
            for (int t = 0; t < kRowBatch; ++t)
                if (p + t < e) dd_accumulate(hi, lo, v[t], xv[t]);
        }
        return hi;
    }
    return bi - row_dot(a.rp, a.ci, a.kval, x, i);
}

// rho = b - K x; partials (buffer 0): ||rho||^2, ||x||^2, ||b||^2, non-finite b flag,
// max |rho_i|, max |x_i|
template <bool kDD>
__global__ void __launch_bounds__(kStreamBlock) k_resid(KrylovArgs a, const double *b, const double *x, double *r) {
    __shared__ double red[kStreamBlock / 64];
    int64_t r0, r1;
    block_rows(a.n, r0, r1);
    double sr = 0.0, sx = 0.0, sb = 0.0, mr = 0.0, mx = 0.0;
    int badb = 0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const double bi = b[i];
        const double ri = resid_row<kDD>(a, x, bi, i);
        r[i] = ri;
        sr += ri * ri;
        sx += x[i] * x[i];
        sb += bi * bi;
        mr = fmax(mr, fabs(ri));
        mx = fmax(mx, fabs(x[i]));
        badb |= !isfinite(bi);
    }
    sr = block_sum(sr, red);
    mr = block_max(mr, red);
    mx = block_max(mx, red);
    sx = block_sum(sx, red);
    sb = block_sum(sb, red);
    const double bad = block_sum((double)badb, red);
    if (threadIdx.x == 0) {
        double *p = partbuf(a, 0) + (int64_t)blockIdx.x * kPartStride;
        p[0] = sr;
        p[1] = sx;
        p[2] = sb;
        p[3] = bad;
        p[4] = mr;
        p[5] = mx;
    }
}

// One block: sums of the residual kernel's partials into the control block.
// The control block starts with the fields of ControlSummary, in the same layout.
static_assert(sizeof(ControlSummary) % 8 == 0 && sizeof(ControlSummary) <= sizeof(Control),
              "ControlSummary is copied as 64-bit words from the start of Control");

// Reduces the residual kernel's partials into the control block, then copies the control
// summary into pinned host memory (system-scope stores: visible to the host once the stream
// has been synchronized), so reading it back needs no separate copy.
__global__ void __launch_bounds__(kStreamBlock) k_resid_reduce(KrylovArgs a, int G, ControlSummary *pub) {
    __shared__ double h[4];
    __shared__ double red[4 * (kStreamBlock / 64)];
    reduce_cols(partbuf(a, 0), G, 4, h, red);
    const double *buf = partbuf(a, 0);
    const int bb = threadIdx.x;
    double mr_t = 0.0, mx_t = 0.0;
    for (int r = bb; r < G; r += kStreamBlock) {
        mr_t = fmax(mr_t, buf[(int64_t)r * kPartStride + 4]);
        mx_t = fmax(mx_t, buf[(int64_t)r * kPartStride + 5]);
    }
    const double mr = block_max(mr_t, red);
    const double mx = block_max(mx_t, red);
    if (threadIdx.x == 0) {
        a.ctl->rinf = mr;
        a.ctl->xinf = mx;
        a.ctl->rnorm2 = h[0];
        a.ctl->xnorm2 = h[1];
        a.ctl->bnorm2 = h[2];
        if (h[3] != 0.0) a.ctl->nonfinite_b = 1;
        // every word loaded first, then stored: one round trip to the control block instead
        // of one per word (a load, its store, the next load ... took 10-16 us per launch)
        constexpr int kWords = sizeof(ControlSummary) / 8;
        const unsigned long long *src = reinterpret_cast<const unsigned long long *>(a.ctl);
        unsigned long long *dst = reinterpret_cast<unsigned long long *>(pub);
        unsigned long long wv[kWords];
#pragma unroll
        for (int w = 0; w < kWords; ++w) wv[w] = src[w];
#pragma unroll
        for (int w = 0; w < kWords; ++w) __hip_atomic_store(dst + w, wv[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Start of a cycle: v_0 = rho / ||rho||, g = (beta, 0, ...), re-arm sentinels
// (and, when xsave is given, xsave = x: the iterate the cycle starts from is the best so far)
template <typename T>
__global__ void __launch_bounds__(kStreamBlock) k_cycle_start(KrylovArgs a, const double *r, double inner_tol,
                                                              T *s1, T *s2, const double *x, double *xsave) {
    const double beta = sqrt(a.ctl->rnorm2);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        a.V[i] = r[i] / beta;
        s1[i] = sentinel<T>();
        s2[i] = sentinel<T>();
        if (xsave) xsave[i] = x[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Control *c = a.ctl;
        c->work_lower = 0;
        c->work_upper = 0;
        c->beta = beta;
        c->inner_tol = inner_tol;
        c->stop = 0;
        c->jdone = 0;
        c->breakdown = 0;
        c->est = beta;
        for (int t = 0; t <= kRestartMax; ++t) c->g[t] = 0.0;
        c->g[0] = beta;
    }
}

// x += Z y with y = H^-1 g (jdone x jdone upper triangular, solved in every block)
__global__ void __launch_bounds__(kStreamBlock) k_xupdate(KrylovArgs a, double *x) {
    __shared__ double y[kRestartMax];
    const Control *c = a.ctl;
    const int m = c->jdone;
    if (threadIdx.x == 0) {
        for (int t = m - 1; t >= 0; --t) {
            double s = c->gr[t];
            for (int u = t + 1; u < m; ++u) {
                const double prod = c->H[u * (kRestartMax + 1) + t] * y[u];
                s = s - prod;
            }
            const double dgn = c->H[t * (kRestartMax + 1) + t];
            y[t] = dgn != 0.0 ? s / dgn : 0.0;
        }
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        double s = x[i];
        for (int t = 0; t < m; ++t) {
            const double prod = a.Z[(int64_t)t * a.n + i] * y[t];
            s = s + prod;
        }
        x[i] = s;
    }
}

// x += d (and, when xsave is given, xsave = x before the update)
__global__ void k_axpy(int64_t n, const double *d, double *x, double *xsave) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        if (xsave) xsave[i] = xi;
        x[i] = xi + d[i];
    }
}

__global__ void k_copy(int64_t n, const double *src, double *dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_widen(int64_t n, const float *src, double *dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------

namespace {

thread_local std::string g_last_error;

struct DevLayout {
    // structure
    int64_t *fp;
    int32_t *fi, *fdiag, *order, *clev, *f2t;
    int64_t *relptr, *fsrc;
    int32_t *relpos, *relsrc, *item, *relslot, *pnu;
    int64_t *pc, *pu;
    uint8_t *item_lane;
    int64_t *krp;
    int32_t *lci, *uci, *kci;
    int32_t *prow, *q;
    // the vector order of a solve: its permutation, the copy of K's entry sources, and the
    // pivot permutations composed with it
    int32_t *vperm, *prow_k, *q_k, *fsrc32;
    int64_t *ostart;
    // triangular-solve schedules (L, U): rows, level starts, lanes, tiles, references
    int32_t *l_rows, *l_seg, *l_tdesc, *l_ref, *l_esrc, *l_src, *l_src_k;
    int32_t *u_rows, *u_seg, *u_tdesc, *u_ref, *u_esrc, *u_q, *u_q_k;
    int64_t *l_rent, *u_rent;
    int32_t *l_sdof, *u_sdof;
    int32_t *l_slg, *u_slg;
    // values
    double *kval, *F64, *T64;
    float *F32, *T32;
    double *Ld64;
    float *Ld32;
    // vectors
    double *V, *Z, *w, *r, *y64, *z64, *dv, *rr, *xb, *bi, *xi;
    float *y32, *z32;
    double *part;
    Control *ctl;
};

}  // namespace

}  // namespace kkt

struct kkt_handle_s {
    size_t tile_lds = kkt::kTileLds;  // dynamic LDS bytes of a solve block (the tile budget)
    kkt_opts_t opts{};
    kkt::Analysis an;
    std::string err;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int device = -1;
    kkt::DevLayout d{};
    bool bound = false;
    bool device_failed = false;
    bool have_factors = false;
    int factor_precision = 0;
    int grid_refactor64 = 0, grid_refactor32 = 0, grid_trsv64 = 0, grid_trsv32 = 0, grid_stream = 0;
    kkt::ControlSummary *host_ctl = nullptr;  // pinned, mapped: written by k_resid_reduce
    kkt::ControlSummary *dev_ctl_sum = nullptr;  // the same memory as seen by kernels
    kkt::StepRecord *host_rec = nullptr;      // pinned, kRestartMax + 1 records (one per step)
    kkt::StepRecord *dev_rec = nullptr;       // the same memory as seen by kernels
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    int restart_alloc = 0;
    bool fp64_current = false;  // mixed mode: FP64 factors of the current system exist
    int64_t repivots = 0;       // re-pivoted factorizations so far
    uint64_t analysis_id = 0;   // identifies the analysis (clones share it; a re-pivot gets a new one)
    uint64_t bind_gen = 0;      // changes at every kkt_bind_workspace (graph cache validity)
    int64_t graph_launches = 0; // refactorizations replayed from a captured graph
    unsigned long long step_token = 0;  // tag of the last Arnoldi step launched
    // per-launch timing (kkt_set_profiling)
    struct ProfRec {
        int cls;
        hipEvent_t a, b;
    };
    uint32_t prof_mask = 0;  // kernel classes timed with events (bit c: class c)
    std::vector<hipEvent_t> ev_pool;
    std::vector<ProfRec> ev_pending;
    kkt_kernel_times_t times{};
};

using kkt::Analysis;

namespace kkt {
namespace {

kkt_status_t fail(kkt_handle_t h, kkt_status_t s, const std::string &m) {
    if (h) h->err = m;
    g_last_error = m;
    return s;
}

#define KKT_HIP(h, call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (h)->device_failed = true;                                                          \
            return fail((h), KKT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
        }                                                                                       \
    } while (0)

// --- per-launch timing with HIP events --------------------------------------------------
hipEvent_t prof_begin(kkt_handle_t h, int cls, hipStream_t s) {
    if (!(h->prof_mask & (1u << cls))) return nullptr;
    hipEvent_t e = nullptr;
    if (!h->ev_pool.empty()) {
        e = h->ev_pool.back();
        h->ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, s) != hipSuccess) {
        h->ev_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void prof_end(kkt_handle_t h, int cls, hipEvent_t a, hipStream_t s) {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (!h->ev_pool.empty()) {
        b = h->ev_pool.back();
        h->ev_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
        h->ev_pool.push_back(a);
        return;
    }
    if (hipEventRecord(b, s) != hipSuccess) {
        h->ev_pool.push_back(a);
        h->ev_pool.push_back(b);
        return;
    }
    h->ev_pending.push_back({cls, a, b});
}

// Accumulates completed records; call after the stream has been synchronized.
void prof_collect(kkt_handle_t h) {
    for (auto &r : h->ev_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            h->times.launches[r.cls] += 1;
            h->times.ms[r.cls] += ms;
        }
        h->ev_pool.push_back(r.a);
        h->ev_pool.push_back(r.b);
    }
    h->ev_pending.clear();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Planner {
    size_t off = 0;
    template <typename T> size_t take(size_t count) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(count, 1) * sizeof(T));
        return o;
    }
};

// Offsets of every array inside the workspace (also gives the total size).
struct Offsets {
    size_t fp, fi, fdiag, order, clev, f2t, relptr, fsrc, relpos, relsrc, relslot, pc, pu, pnu, item, item_lane, krp, kci, l_rows, l_seg, l_tdesc,
        l_ref, l_slg, l_esrc, l_rent, l_sdof, l_src, l_src_k, u_rows, u_seg, u_tdesc, u_ref, u_slg, u_esrc,
        u_rent, u_sdof, u_q, u_q_k, prow, q, vperm, prow_k, q_k, ostart, fsrc32, kval, F64, T64, F32, T32, Ld64, Ld32, V, Z, w, r, y64, z64, y32,
        z32, dv, rr, xb, bi, xi, part, ctl, total;
};

Offsets plan(const kkt_handle_t h) {
    const Analysis &a = h->an;
    const int64_t n = a.n, f = a.nnz_f();
    const int R = h->opts.restart;
    Planner p;
    Offsets o{};
    o.fp = p.take<int64_t>(n + 1);
    o.fi = p.take<int32_t>(f);
    o.fdiag = p.take<int32_t>(n);
    o.order = p.take<int32_t>(n);
    o.clev = p.take<int32_t>(n);
    o.f2t = p.take<int32_t>(f);
    o.relptr = p.take<int64_t>(n + 1);
    // F positions' value sources: 32-bit for the flat refactorization (which reads them), 64-bit
    // for the other one (whose ingest initializes F)
    o.fsrc = p.take<int64_t>(a.phys ? 0 : f);
    o.fsrc32 = p.take<int32_t>(a.phys ? f : 0);
    o.relpos = p.take<int32_t>(a.relpos.size());
    o.relsrc = p.take<int32_t>(a.relsrc.size());
    o.relslot = p.take<int32_t>(a.relslot.size());
    o.pc = p.take<int64_t>(a.pc.size());
    o.pu = p.take<int64_t>(a.pu.size());
    o.pnu = p.take<int32_t>(a.pnu.size());
    o.item = p.take<int32_t>(a.ref_item.size());
    o.item_lane = p.take<uint8_t>(a.ref_item_lane.size());
    o.krp = p.take<int64_t>(n + 1);
    o.kci = p.take<int32_t>(a.nnz);
    o.l_rows = p.take<int32_t>(n);
    o.l_seg = p.take<int32_t>(a.lsched.seg_row.size());
    o.l_tdesc = p.take<int32_t>(kTileDesc * a.lsched.tiles());
    o.l_src = p.take<int32_t>(n);
    o.l_src_k = p.take<int32_t>(n);
    o.l_ref = p.take<int32_t>(a.lsched.ent_ref.size());
    o.l_esrc = p.take<int32_t>(a.lsched.ext_src.size());
    o.l_rent = p.take<int64_t>(a.lsched.row_ent.size());
    o.l_sdof = p.take<int32_t>(a.lsched.seg_dofs.size());
    o.l_slg = p.take<int32_t>(a.lsched.seg_lg.size());
    o.u_rows = p.take<int32_t>(n);
    o.u_seg = p.take<int32_t>(a.usched.seg_row.size());
    o.u_tdesc = p.take<int32_t>(kTileDesc * a.usched.tiles());
    o.u_q = p.take<int32_t>(n);
    o.u_q_k = p.take<int32_t>(n);
    o.u_ref = p.take<int32_t>(a.usched.ent_ref.size());
    o.u_esrc = p.take<int32_t>(a.usched.ext_src.size());
    o.u_rent = p.take<int64_t>(a.usched.row_ent.size());
    o.u_sdof = p.take<int32_t>(a.usched.seg_dofs.size());
    o.u_slg = p.take<int32_t>(a.usched.seg_lg.size());
    o.prow = p.take<int32_t>(n);
    o.q = p.take<int32_t>(n);
    o.vperm = p.take<int32_t>(n);
    o.prow_k = p.take<int32_t>(n);
    o.q_k = p.take<int32_t>(n);
    o.ostart = p.take<int64_t>(n);
    o.kval = p.take<double>(a.nnz);
    o.F64 = p.take<double>(f);
    o.T64 = p.take<double>(a.t_size);
    o.F32 = p.take<float>(f);
    o.T32 = p.take<float>(a.t_size);
    o.Ld64 = p.take<double>(f);
    o.Ld32 = p.take<float>(f);
    o.V = p.take<double>((size_t)(R + 1) * n);
    o.Z = p.take<double>((size_t)R * n);
    o.w = p.take<double>(n);
    o.r = p.take<double>(n);
    o.y64 = p.take<double>(n);
    o.z64 = p.take<double>(n);
    o.y32 = p.take<float>(n);
    o.z32 = p.take<float>(n);
    o.dv = p.take<double>(n);
    o.rr = p.take<double>(n);
    o.xb = p.take<double>(n);
    o.bi = p.take<double>(n);
    o.xi = p.take<double>(n);
    o.part = p.take<double>((size_t)3 * kStreamGridMax * kPartStride);
    o.ctl = p.take<Control>(1);
    o.total = p.off;
    return o;
}

template <typename T> hipError_t up(char *base, size_t off, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Per-tile descriptors of a solve schedule (kTileDesc ints each, the layout k_trsv reads).
std::vector<int32_t> tile_descriptors(const TriSchedule &sc) {
    std::vector<int32_t> d((size_t)kTileDesc * sc.tiles(), 0);
    for (int64_t t = 0; t < sc.tiles(); ++t) {
        int32_t *x = d.data() + kTileDesc * t;
        const int32_t s0 = sc.tile_seg[t], s1 = sc.tile_seg[t + 1];
        const int32_t rb = sc.seg_row[s0], re = sc.seg_row[s1];
        const int64_t eb = sc.row_ent[rb], db = sc.tile_dense[t];
        x[0] = s0;
        x[1] = s1;
        x[2] = rb;
        x[3] = re;
        x[4] = (int32_t)(uint32_t)(uint64_t)eb;
        x[5] = (int32_t)(uint32_t)((uint64_t)eb >> 32);
        x[6] = (int32_t)(sc.row_ent[re] - eb);
        x[7] = sc.tile_ext[t];
        x[8] = sc.tile_ext[t + 1] - sc.tile_ext[t];
        x[9] = (int32_t)(uint32_t)(uint64_t)db;
        x[10] = (int32_t)(uint32_t)((uint64_t)db >> 32);
        x[11] = (int32_t)(sc.tile_dense[t + 1] - db);
        x[12] = sc.tile_lds[t];
    }
    return d;
}

// Blocks of 256 threads that fit on the device at once (a persistent grid size).
int coop_grid(const void *func, int device, size_t dyn_lds = 0) {
    int per_cu = 0, cus = 0;
    if (dyn_lds > 0 &&
        hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, kCoopBlock, dyn_lds) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

template <typename T> KrylovArgs kargs(kkt_handle_t h) {
    KrylovArgs k;
    k.n = h->an.n;
    k.rp = h->d.krp;
    k.ci = h->d.kci;
    k.kval = h->d.kval;
    k.V = h->d.V;
    k.Z = h->d.Z;
    k.w = h->d.w;
    k.part = h->d.part;
    k.ctl = h->d.ctl;
    return k;
}

// Blocks of 256 threads for the row-wise ingest: one row per thread up to 4,096 blocks (its
// rows' loads are two dependent rounds, so more rows in flight hide their latency).
int ingest_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

int stream_blocks(int64_t n) {
    int64_t b = (n + kStreamBlock - 1) / kStreamBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kStreamGridMax));
}

template <typename T>
// vorder: the right-hand side and the solution are in the vector order of a solve (else in
// the caller's original order)
hipError_t launch_trsv(kkt_handle_t h, bool lower, const double *rhs64, const T *rhs_step, T *out, double *xout,
                       const Control *stopflag, hipStream_t s, bool vorder, unsigned int *work = nullptr,
                       unsigned int *hang = nullptr) {
    const Analysis &a = h->an;
    TrsvArgs<T> t{};
    const bool is64 = sizeof(T) == 8;
    const TriSchedule &sc = lower ? a.lsched : a.usched;
    t.ntiles = sc.tiles();
    const DevLayout &d = h->d;
    t.seg_row = lower ? d.l_seg : d.u_seg;
    t.seg_lg = lower ? d.l_slg : d.u_slg;
    t.rows = lower ? d.l_rows : d.u_rows;
    t.row_ent = lower ? d.l_rent : d.u_rent;
    t.ent_ref = lower ? d.l_ref : d.u_ref;
    t.ext_src = lower ? d.l_esrc : d.u_esrc;
    t.tdesc = lower ? d.l_tdesc : d.u_tdesc;
    t.seg_dofs = lower ? d.l_sdof : d.u_sdof;
    const T *base = (const T *)(is64 ? (void *)d.T64 : (void *)d.T32);
    if (lower) {
        t.val = base;
        t.rhs64 = rhs64;
        t.rsrc = vorder ? d.l_src_k : d.l_src;
    } else {
        t.val = base + a.lsched.values();
        t.diag = base + a.lsched.values() + a.usched.values();
        t.rhs_step = rhs_step;
        t.xout = xout;
        t.qpos = vorder ? d.u_q_k : d.u_q;
    }
    t.out = out;
    t.stopflag = stopflag;
    t.work = work ? work : lower ? &d.ctl->work_lower : &d.ctl->work_upper;
    t.hang = hang ? hang : &d.ctl->hang;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(is64 ? h->grid_trsv64 : h->grid_trsv32, t.ntiles));
    // the variant without the dense-segment path when the schedule has none
    const bool dense = sc.values() > sc.packed;
    if (lower && dense) k_trsv<T, true, true><<<grid, kTileThreads, h->tile_lds, s>>>(t);
    else if (lower) k_trsv<T, true, false><<<grid, kTileThreads, h->tile_lds, s>>>(t);
    else if (dense) k_trsv<T, false, true><<<grid, kTileThreads, h->tile_lds, s>>>(t);
    else k_trsv<T, false, false><<<grid, kTileThreads, h->tile_lds, s>>>(t);
    return hipGetLastError();
}

// x = Q U^-1 L^-1 P b with the current factors of precision T (sentinels armed before); b and
// x in the vector order of a solve (vorder) or in the original order.
template <typename T>
hipError_t precond(kkt_handle_t h, const double *b, double *x, const Control *ctl, hipStream_t s, bool vorder) {
    T *y = (T *)(sizeof(T) == 8 ? (void *)h->d.y64 : (void *)h->d.y32);
    T *z = (T *)(sizeof(T) == 8 ? (void *)h->d.z64 : (void *)h->d.z32);
    hipEvent_t e0 = prof_begin(h, KKT_K_TRSV_L, s);
    hipError_t e = launch_trsv<T>(h, true, b, nullptr, y, nullptr, ctl, s, vorder);
    prof_end(h, KKT_K_TRSV_L, e0, s);
    if (e != hipSuccess) return e;
    e0 = prof_begin(h, KKT_K_TRSV_U, s);
    e = launch_trsv<T>(h, false, nullptr, y, z, x, ctl, s, vorder);
    prof_end(h, KKT_K_TRSV_U, e0, s);
    return e;
}

template <typename T> void rearm(kkt_handle_t h, hipStream_t s) {
    T *y = (T *)(sizeof(T) == 8 ? (void *)h->d.y64 : (void *)h->d.y32);
    T *z = (T *)(sizeof(T) == 8 ? (void *)h->d.z64 : (void *)h->d.z32);
    hipEvent_t e0 = prof_begin(h, KKT_K_OTHER, s);
    k_fill_sentinel<T><<<h->grid_stream, kStreamBlock, 0, s>>>(h->an.n, y, z, &h->d.ctl->work_lower,
                                                                &h->d.ctl->work_upper, nullptr);
    prof_end(h, KKT_K_OTHER, e0, s);
}

// Enqueues ingest + numeric refactorization of `count` systems of one pattern: handle hs[b]
// (bound to the same analysis as hs[0]) gets the values at vals[b] (device; when null, the
// values already in its workspace are re-ingested).  Ingest runs per system; the
// refactorizations of all of them run in one launch, with hs[0]'s structure arrays.
kkt_status_t refactor_batch_impl(const kkt_handle_t *hs, const double *const *vals, int count, int precision,
                                 hipStream_t s) {
    const kkt_handle_t h = hs[0];
    const Analysis &a = h->an;
    const int64_t f = a.nnz_f();
    auto fail_all = [&](const std::string &m) {
        for (int b = 0; b < count; ++b) hs[b]->device_failed = true;
        for (int b = 1; b < count; ++b) fail(hs[b], KKT_EDEVICE, m);
        return fail(h, KKT_EDEVICE, m);
    };
    hipEvent_t e0 = prof_begin(h, KKT_K_INGEST, s);
    for (int b = 0; b < count; ++b) {
        DevLayout &d = hs[b]->d;
        if (vals[b]) {
            k_prep_values<<<1, 1, 0, s>>>(d.ctl);
            k_ingest_rows<<<ingest_grid(a.n), 256, 0, s>>>(a.n, d.ostart, d.krp, vals[b], d.kval, d.ctl);
        }
        k_prep_refactor<<<1, 1, 0, s>>>(d.ctl);
        k_arm<<<2048, 256, 0, s>>>(f, a.phys ? nullptr : d.fsrc, d.kval, d.F64, d.F32, d.Ld64, d.Ld32, precision);
    }
    prof_end(h, KKT_K_INGEST, e0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_all(std::string("ingest: ") + hipGetErrorString(e));
    e0 = prof_begin(h, KKT_K_REFACTOR, s);
    const DevLayout &d = h->d;
    const int64_t nitems = (int64_t)a.ref_item.size() - 1;
    if (precision == KKT_PREC_MIXED) {
        RefactorArgs<float> r{a.n, d.fp, d.fi, d.fdiag, d.relptr, d.relpos, d.order, d.clev, d.f2t, d.relsrc,
                              d.relslot, d.pc, d.pu, d.pnu, d.fsrc32, d.kval, d.item, d.item_lane, nitems, d.F32,
                              d.T32, d.Ld32,
                              h->opts.guard_policy,
                              d.ctl};
        RefactorBatch<float> bt{};
        bt.nslots = count;
        for (int b = 0; b < count; ++b)
            bt.slot[b] = {hs[b]->d.F32, hs[b]->d.T32, hs[b]->d.Ld32, hs[b]->d.ctl, hs[b]->d.kval};
        if (!a.relsrc.empty()) k_refactor<float, true><<<h->grid_refactor32, kCoopBlock, 0, s>>>(r, bt);
        else k_refactor<float, false><<<h->grid_refactor32, kCoopBlock, 0, s>>>(r, bt);
    } else {
        RefactorArgs<double> r{a.n, d.fp, d.fi, d.fdiag, d.relptr, d.relpos, d.order, d.clev, d.f2t, d.relsrc,
                               d.relslot, d.pc, d.pu, d.pnu, d.fsrc32, d.kval, d.item, d.item_lane, nitems, d.F64,
                               d.T64, d.Ld64,
                               h->opts.guard_policy,
                               d.ctl};
        RefactorBatch<double> bt{};
        bt.nslots = count;
        for (int b = 0; b < count; ++b)
            bt.slot[b] = {hs[b]->d.F64, hs[b]->d.T64, hs[b]->d.Ld64, hs[b]->d.ctl, hs[b]->d.kval};
        if (!a.relsrc.empty()) k_refactor<double, true><<<h->grid_refactor64, kCoopBlock, 0, s>>>(r, bt);
        else k_refactor<double, false><<<h->grid_refactor64, kCoopBlock, 0, s>>>(r, bt);
    }
    prof_end(h, KKT_K_REFACTOR, e0, s);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_all(std::string("refactorization: ") + hipGetErrorString(e));
    for (int b = 0; b < count; ++b) {
        hs[b]->have_factors = true;
        hs[b]->factor_precision = precision;
    }
    return KKT_OK;
}

kkt_status_t refactor_impl(kkt_handle_t h, const double *dev_values, int precision, hipStream_t s) {
    return refactor_batch_impl(&h, &dev_values, 1, precision, s);
}

void launch_resid(kkt_handle_t h, const KrylovArgs &ka, const double *b, const double *x, double *r, hipStream_t s) {
    if (h->opts.residual == KKT_RESID_DD) k_resid<true><<<h->grid_stream, kStreamBlock, 0, s>>>(ka, b, x, r);
    else k_resid<false><<<h->grid_stream, kStreamBlock, 0, s>>>(ka, b, x, r);
}

// The summary is already in host memory (k_resid_reduce wrote it): wait for the stream.
kkt_status_t read_ctl(kkt_handle_t h, hipStream_t s) {
    KKT_HIP(h, hipStreamSynchronize(s));
    prof_collect(h);
    if (h->host_ctl->hang) {
        h->device_failed = true;
        return fail(h, KKT_EDEVICE, "a dependency wait exceeded its spin limit");
    }
    return KKT_OK;
}

// One FGMRES-IR solve with the factors currently in the workspace (Section 2.1): x0 from
// the direct solve, the refine test of Section 2.3, then restart cycles whose solution is
// formed only at the end of the cycle.  The host reads each Arnoldi step's stop flag while
// the next step runs; at most one step is enqueued past the end of a cycle, and its kernels
// return at once.
// require_nrbe = false runs FGMRES as an inner solver (acceptance on its estimate only).
template <typename T>
kkt_status_t solve_impl(kkt_handle_t h, const double *b, double *x, double tol, kkt_solve_info_t *info,
                        hipStream_t s, int max_cycles, bool require_nrbe = true) {
    const Analysis &a = h->an;
    DevLayout &d = h->d;
    const int R = h->opts.restart;
    const int G = h->grid_stream;
    KrylovArgs ka = kargs<T>(h);
    T *y = (T *)(sizeof(T) == 8 ? (void *)d.y64 : (void *)d.y32);
    T *z = (T *)(sizeof(T) == 8 ? (void *)d.z64 : (void *)d.z32);
    hipEvent_t e0 = prof_begin(h, KKT_K_OTHER, s);
    k_prep_solve<<<1, 1, 0, s>>>(d.ctl);
    prof_end(h, KKT_K_OTHER, e0, s);
    rearm<T>(h, s);
    KKT_HIP(h, precond<T>(h, b, x, nullptr, s, true));
    e0 = prof_begin(h, KKT_K_RESID, s);
    launch_resid(h, ka, b, x, d.r, s);
    k_resid_reduce<<<1, kStreamBlock, 0, s>>>(ka, G, h->dev_ctl_sum);
    prof_end(h, KKT_K_RESID, e0, s);
    KKT_HIP(h, hipGetLastError());
    kkt_status_t st = read_ctl(h, s);
    if (st != KKT_OK) return st;
    const ControlSummary &c = *h->host_ctl;
    if (c.nonfinite) return fail(h, KKT_EINVAL, "non-finite value in the matrix of the last refactorization");
    if (c.nonfinite_b) return fail(h, KKT_EINVAL, "non-finite value in the right-hand side");
    if (c.guard_fail) return fail(h, KKT_ESINGULAR, "tiny static pivot under the FAIL guard policy");
    double knorm;
    {
        unsigned long long bits = c.knorm_bits;
        std::memcpy(&knorm, &bits, sizeof(knorm));
    }
    const double bn = std::sqrt(c.bnorm2);
    const double rho0 = std::sqrt(c.rnorm2);
    double rn = rho0;
    double nrbe = rn / (knorm * std::sqrt(c.xnorm2) + bn);
    kkt_solve_info_t inf{};
    inf.precision = sizeof(T) == 8 ? KKT_PREC_FP64 : KKT_PREC_MIXED;
    inf.pivots_perturbed = (int64_t)c.nguard;
    inf.knorm_inf = knorm;
    inf.precond_applications = 1;
    inf.nrbe0 = nrbe;
    const bool paper = h->opts.stop_mode == KKT_STOP_PAPER;
    const double target = require_nrbe ? h->opts.nrbe_target : HUGE_VAL;
    bool converged;
    if (bn == 0.0) converged = true;
    else converged = paper ? (rn / bn < tol && nrbe <= target) : nrbe <= target;
    inf.refined = !converged;
    int iters = 0, cycles = 0;
    double est = rn;
    // The iterate with the lowest true residual so far (x0 included) is what a solve that
    // does not converge returns.  x holds it while x_best; a cycle that starts from it saves
    // a copy in xb first (fused into the cycle start), and its summary is kept for the info.
    const bool track = require_nrbe;
    bool x_best = true;
    double best_rn = rho0;
    ControlSummary best_sum = c;
    while (!converged && cycles < max_cycles) {
        ++cycles;
        if (!(rn > 0.0)) {
            converged = true;
            break;
        }
        const double xn = std::sqrt(h->host_ctl->xnorm2);
        const double inner = paper ? tol * rho0 : target * (knorm * xn + bn);
        e0 = prof_begin(h, KKT_K_OTHER, s);
        const bool save = track && x_best;
        k_cycle_start<T><<<G, kStreamBlock, 0, s>>>(ka, d.r, inner, y, z, save ? x : nullptr,
                                                      save ? d.xb : nullptr);
        prof_end(h, KKT_K_OTHER, e0, s);
        // Step j+1 is enqueued before the host reads step j's record, so the device never
        // waits for the host; kernels of a step enqueued after the stop return at once.
        // DCGS2 takes one step more: step R only finishes column R - 1.
        const bool dcgs2 = h->opts.gram_schmidt == KKT_GS_DCGS2;
        const int steps = dcgs2 ? R + 1 : R;
        for (int j = 0; j < steps; ++j) {
            const size_t step_mark = h->ev_pending.size();
            if (j < R) KKT_HIP(h, precond<T>(h, d.V + (int64_t)j * a.n, d.Z + (int64_t)j * a.n, d.ctl, s, true));
            e0 = prof_begin(h, KKT_K_SPMV, s);
            if (dcgs2) k_dcgs2_dots<<<G, kStreamBlock, 0, s>>>(ka, j, j < R ? 1 : 0);
            else k_spmv_dots<<<G, kStreamBlock, 0, s>>>(ka, j);
            prof_end(h, KKT_K_SPMV, e0, s);
            e0 = prof_begin(h, KKT_K_CGS, s);
            const unsigned long long token = ++h->step_token;
            if (dcgs2) {
                k_dcgs2<T><<<G, kStreamBlock, 0, s>>>(ka, j, R, y, z, h->dev_rec, token);
            } else {
                k_cgs_pass2<<<G, kStreamBlock, 0, s>>>(ka, j);
                k_cgs_finish<<<G, kStreamBlock, 0, s>>>(ka, j);
                k_normalize<T><<<G, kStreamBlock, 0, s>>>(ka, j, R, y, z, h->dev_rec, token);
            }
            prof_end(h, KKT_K_CGS, e0, s);
            KKT_HIP(h, hipGetLastError());
            KKT_HIP(h, hipEventRecord(h->step_ev[j & 1], s));
            if (j == 0) continue;
            KKT_HIP(h, hipEventSynchronize(h->step_ev[(j - 1) & 1]));
            // the record of step j - 1 carries the token it was launched with; until it shows,
            // the slot may still hold an older step's record, so wait for it (bounded, then
            // fall back to a full synchronization)
            StepRecord &rec = h->host_rec[j - 1];
            const unsigned long long want = h->step_token - 1;
            bool seen = false;
            for (int spin = 0; spin < (1 << 20) && !seen; ++spin)
                seen = __atomic_load_n(&rec.token, __ATOMIC_ACQUIRE) == want;
            if (!seen) {
                KKT_HIP(h, hipStreamSynchronize(s));
                seen = __atomic_load_n(&rec.token, __ATOMIC_ACQUIRE) == want;
                if (!seen) {
                    h->device_failed = true;
                    return fail(h, KKT_EDEVICE, "an Arnoldi step record did not arrive");
                }
            }
            if (rec.hang) {
                h->device_failed = true;
                return fail(h, KKT_EDEVICE, "a dependency wait exceeded its spin limit");
            }
            if (rec.stop) {
                // step j does no work: its timing records are not kept
                for (size_t q = step_mark; q < h->ev_pending.size(); ++q) {
                    h->ev_pool.push_back(h->ev_pending[q].a);
                    h->ev_pool.push_back(h->ev_pending[q].b);
                }
                h->ev_pending.resize(step_mark);
                break;
            }
        }
        e0 = prof_begin(h, KKT_K_OTHER, s);
        k_xupdate<<<G, kStreamBlock, 0, s>>>(ka, x);
        prof_end(h, KKT_K_OTHER, e0, s);
        e0 = prof_begin(h, KKT_K_RESID, s);
        launch_resid(h, ka, b, x, d.r, s);
        k_resid_reduce<<<1, kStreamBlock, 0, s>>>(ka, G, h->dev_ctl_sum);
        prof_end(h, KKT_K_RESID, e0, s);
        KKT_HIP(h, hipGetLastError());
        st = read_ctl(h, s);
        if (st != KKT_OK) return st;
        iters += h->host_ctl->jdone;
        // a DCGS2 cycle that stops before its last step has applied M^-1 once more
        inf.precond_applications += h->host_ctl->jdone + (dcgs2 && h->host_ctl->jdone < R ? 1 : 0);
        est = h->host_ctl->est;
        rn = std::sqrt(h->host_ctl->rnorm2);
        nrbe = rn / (knorm * std::sqrt(h->host_ctl->xnorm2) + bn);
        // NRBE alone is lenient when ||x|| grows (||K|| ||x|| is in its denominator): an
        // iterate whose true residual exceeds that of x0 is never accepted
        converged = (paper ? (est < tol * rho0 && nrbe <= target) : nrbe <= target) && rn <= rho0;
        x_best = rn < best_rn;
        if (x_best) {
            best_rn = rn;
            best_sum = *h->host_ctl;
        }
    }
    const ControlSummary *fin = h->host_ctl;
    if (!converged && track && !x_best) {
        // restore the best iterate (saved when the cycle that left it started)
        e0 = prof_begin(h, KKT_K_OTHER, s);
        k_copy<<<G, kStreamBlock, 0, s>>>(a.n, d.xb, x);
        prof_end(h, KKT_K_OTHER, e0, s);
        KKT_HIP(h, hipGetLastError());
        fin = &best_sum;
        rn = best_rn;
        nrbe = rn / (knorm * std::sqrt(fin->xnorm2) + bn);
        inf.restored_best = 1;
    }
    inf.converged = converged;
    inf.iterations = iters;
    inf.cycles = cycles;
    inf.nrbe = nrbe;
    inf.rel_resid = bn > 0.0 ? rn / bn : 0.0;
    inf.rr = rho0 > 0.0 ? rn / rho0 : 0.0;
    inf.est_resid = est;
    inf.true_resid = rn;
    inf.nsr = fin->rinf / (knorm * fin->xinf);
    if (info) *info = inf;
    return converged ? KKT_OK : KKT_ENOCONV;
}

// Richardson iterative refinement (Section 1.3), optionally with each correction computed
// by FGMRES on the error system K d = rho (Section 2.1).  Stops when ||rho|| < tol ||rho0||
// and NRBE <= target, when MA57's ratio test fails (NSR_new > ratio * NSR_old), or after
// richardson_max_it corrections.
template <typename T>
kkt_status_t richardson_impl(kkt_handle_t h, const double *b, double *x, double tol, kkt_solve_info_t *info,
                             hipStream_t s, bool inner_fgmres) {
    const Analysis &a = h->an;
    DevLayout &d = h->d;
    const int G = h->grid_stream;
    KrylovArgs ka = kargs<T>(h);
    hipEvent_t e0 = prof_begin(h, KKT_K_OTHER, s);
    k_prep_solve<<<1, 1, 0, s>>>(d.ctl);
    prof_end(h, KKT_K_OTHER, e0, s);
    rearm<T>(h, s);
    KKT_HIP(h, precond<T>(h, b, x, nullptr, s, true));
    auto residual = [&]() -> kkt_status_t {
        hipEvent_t r0 = prof_begin(h, KKT_K_RESID, s);
        launch_resid(h, ka, b, x, d.r, s);
        k_resid_reduce<<<1, kStreamBlock, 0, s>>>(ka, G, h->dev_ctl_sum);
        prof_end(h, KKT_K_RESID, r0, s);
        KKT_HIP(h, hipGetLastError());
        return read_ctl(h, s);
    };
    kkt_status_t st = residual();
    if (st != KKT_OK) return st;
    const ControlSummary &c = *h->host_ctl;
    if (c.nonfinite) return fail(h, KKT_EINVAL, "non-finite value in the matrix of the last refactorization");
    if (c.nonfinite_b) return fail(h, KKT_EINVAL, "non-finite value in the right-hand side");
    if (c.guard_fail) return fail(h, KKT_ESINGULAR, "tiny static pivot under the FAIL guard policy");
    double knorm;
    {
        unsigned long long bits = c.knorm_bits;
        std::memcpy(&knorm, &bits, sizeof(knorm));
    }
    const double bn = std::sqrt(c.bnorm2);
    const double rho0 = std::sqrt(c.rnorm2);
    double rn = rho0;
    double nrbe = rn / (knorm * std::sqrt(c.xnorm2) + bn);
    double nsr = c.rinf / (knorm * c.xinf);
    kkt_solve_info_t inf{};
    inf.precision = sizeof(T) == 8 ? KKT_PREC_FP64 : KKT_PREC_MIXED;
    inf.pivots_perturbed = (int64_t)c.nguard;
    inf.knorm_inf = knorm;
    inf.nrbe0 = nrbe;
    inf.precond_applications = 1;
    const double target = h->opts.nrbe_target;
    bool converged = bn == 0.0 || (rn < tol * rho0 && nrbe <= target);
    inf.refined = !converged;
    int it = 0;
    // best iterate so far, as in solve_impl: x holds it while x_best, else xb does
    bool x_best = true;
    double best_rn = rho0;
    ControlSummary best_sum = c;
    while (!converged && it < h->opts.richardson_max_it) {
        if (inner_fgmres) {
            hipEvent_t c0 = prof_begin(h, KKT_K_OTHER, s);
            k_copy<<<G, kStreamBlock, 0, s>>>(a.n, d.r, d.rr);
            prof_end(h, KKT_K_OTHER, c0, s);
            kkt_solve_info_t in{};
            st = solve_impl<T>(h, d.rr, d.dv, h->opts.inner_tol, &in, s, 1, false);
            if (st != KKT_OK && st != KKT_ENOCONV) return st;
            inf.precond_applications += in.precond_applications;
            inf.iterations += in.iterations;
        } else {
            rearm<T>(h, s);
            KKT_HIP(h, precond<T>(h, d.r, d.dv, nullptr, s, true));
            inf.precond_applications += 1;
        }
        hipEvent_t x0 = prof_begin(h, KKT_K_OTHER, s);
        k_axpy<<<G, kStreamBlock, 0, s>>>(a.n, d.dv, x, x_best ? d.xb : nullptr);
        prof_end(h, KKT_K_OTHER, x0, s);
        ++it;
        st = residual();
        if (st != KKT_OK) return st;
        rn = std::sqrt(h->host_ctl->rnorm2);
        nrbe = rn / (knorm * std::sqrt(h->host_ctl->xnorm2) + bn);
        const double nsr_new = h->host_ctl->rinf / (knorm * h->host_ctl->xinf);
        converged = rn < tol * rho0 && nrbe <= target;
        x_best = rn < best_rn;
        if (x_best) {
            best_rn = rn;
            best_sum = *h->host_ctl;
        }
        const bool stalled = nsr_new > h->opts.ratio_stop * nsr;
        nsr = nsr_new;
        if (stalled) break;
    }
    if (!converged && !x_best) {
        hipEvent_t x0 = prof_begin(h, KKT_K_OTHER, s);
        k_copy<<<G, kStreamBlock, 0, s>>>(a.n, d.xb, x);
        prof_end(h, KKT_K_OTHER, x0, s);
        KKT_HIP(h, hipGetLastError());
        rn = best_rn;
        nrbe = rn / (knorm * std::sqrt(best_sum.xnorm2) + bn);
        nsr = best_sum.rinf / (knorm * best_sum.xinf);
        inf.restored_best = 1;
    }
    inf.converged = converged;
    inf.cycles = it;
    if (!inner_fgmres) inf.iterations = it;
    inf.nrbe = nrbe;
    inf.nsr = nsr;
    inf.rel_resid = bn > 0.0 ? rn / bn : 0.0;
    inf.rr = rho0 > 0.0 ? rn / rho0 : 0.0;
    inf.est_resid = rn;
    inf.true_resid = rn;
    if (info) *info = inf;
    return converged ? KKT_OK : KKT_ENOCONV;
}

}  // namespace
}  // namespace kkt

// ---------------------------------------------------------------------------------------
// Scratch of the allocation-free direct solve (kkt_direct_solve_noalloc): the two tile
// counters and the wait-failure flag in the first 256 bytes, then the intermediate vectors
// y = L^-1 P b and z = U^-1 y, kNoAllocMaxRows values of 8 bytes each (FP32 factors use the
// first half of each).  One copy per GPU, for the life of the process; calls on one GPU
// share it.
// ---------------------------------------------------------------------------------------

namespace kkt {
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 21;  // 2,097,152 rows
constexpr size_t kNoAllocHead = 256;
constexpr size_t kNoAllocBytes = kNoAllocHead + 2 * sizeof(double) * (size_t)kNoAllocMaxRows;  // 32 MiB + 256 B
struct NoAllocHead {
    unsigned int work_lower, work_upper, hang;
};
}  // namespace kkt

static __device__ __align__(256) unsigned char scratch[kkt::kNoAllocBytes];

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------

using namespace kkt;

namespace kkt {
namespace {

uint64_t next_analysis_id() {
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

AnalysisOptions analysis_options(const kkt_opts_t &o, int64_t n) {
    AnalysisOptions ao;
    ao.ordering = o.ordering == KKT_ORDER_ND ? ORDER_ND : ORDER_MD;
    ao.nd_leaf = o.nd_leaf;
    ao.pivot_tau = o.pivot_tau;
    ao.tile_threads = kTileThreads;
    ao.tile_rows = kTileRows;
    ao.tile_lds = o.tile_lds_kib > 0 ? o.tile_lds_kib * 1024 : kTileLds;
    ao.dense_reserve_l = ao.tile_lds / 2;  // half the tile for dense blocks (60k L solve 123.9 -> 119.7 us against a quarter)
    // Wide levels run as lane items (64 short columns, one per lane) and chunks, narrow ones a
    // column per wavefront.  A lane walks its column's updates alone, which pays while a level
    // has many more columns than there are wavefronts; a level that one wavefront per column
    // covers in a single round is faster on the one-column path.  Hence at least the resident
    // wavefronts of the refactorization (3 blocks of 4 per compute unit, 256 compute units),
    // and n/64 up to 16,384 beyond that: measured best at 60k (3,072: 187 -> 145 us), 500k
    // (~8,192-12,288) and 2M (16,384) unknowns.
    ao.narrow_columns = o.narrow_columns > 0
                            ? o.narrow_columns
                            : (int)std::max<int64_t>(kResidentRefactorWaves, std::min<int64_t>(16384, n / 64));
    return ao;
}

// The pivot sequence of an earlier system no longer suits the current one: repeat the
// threshold-pivoted factorization on the host with the current values (ordering kept), rebuild
// the schedules into the bound workspace and refactor (Section 1.3 describes the first
// system's pivoted factorization; this repeats it for the current one).
kkt_status_t repivot_impl(kkt_handle_t h, hipStream_t s) {
    const Analysis &old = h->an;
    // the workspace's copy of K is in the vector order: back to the original CSR order
    std::vector<double> kv(old.nnz), vals(old.nnz);
    KKT_HIP(h, hipMemcpyAsync(kv.data(), h->d.kval, old.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    KKT_HIP(h, hipStreamSynchronize(s));
    for (int64_t e = 0; e < old.nnz; ++e) vals[old.ksrc[e]] = kv[e];
    AnalysisOptions ao = analysis_options(h->opts, old.n);
    const std::vector<int32_t> q = old.q;
    ao.fixed_order = q.data();
    Analysis na;
    std::string msg;
    const int rc = analyze(ao, old.n, old.rowptr.data(), old.colidx.data(), vals.data(), na, &msg);
    if (rc != AN_OK)
        return fail(h, rc == AN_ESINGULAR ? KKT_ESINGULAR : KKT_EINVAL, "re-pivoting: " + msg);
    Analysis keep = std::move(h->an);
    h->an = std::move(na);
    const uint64_t keep_id = h->analysis_id;
    h->analysis_id = next_analysis_id();
    const size_t need = plan(h).total;
    if (need > h->ws_bytes) {
        h->an = std::move(keep);
        h->analysis_id = keep_id;
        return fail(h, KKT_ENOMEM, "re-pivoting needs a workspace of " + std::to_string(need) + " bytes, " +
                                       std::to_string(h->ws_bytes) + " are bound");
    }
    kkt_status_t st = kkt_bind_workspace(h, h->ws, h->ws_bytes, s);
    if (st != KKT_OK) return st;
    for (int64_t e = 0; e < h->an.nnz; ++e) kv[e] = vals[h->an.ksrc[e]];
    KKT_HIP(h, hipMemcpyAsync(h->d.kval, kv.data(), h->an.nnz * sizeof(double), hipMemcpyHostToDevice, s));
    KKT_HIP(h, hipStreamSynchronize(s));
    k_prep_values<<<1, 1, 0, s>>>(h->d.ctl);
    k_rownorm<<<(int)std::max<int64_t>(1, std::min<int64_t>((h->an.n + 255) / 256, 1024)), 256, 0, s>>>(
        h->an.n, h->d.krp, h->d.kval, h->d.ctl);
    KKT_HIP(h, hipGetLastError());
    // mixed precision: the FP32 factors of the old layout are meaningless now, so the FP32
    // refactorization runs in the new layout as well (kkt_direct_solve and the factor getters
    // read them); the FP64 factors, refactored last, serve this system's remaining solves
    if (h->opts.precision == KKT_PREC_MIXED) {
        st = refactor_impl(h, nullptr, KKT_PREC_MIXED, s);
        if (st != KKT_OK) return st;
    }
    st = refactor_impl(h, nullptr, KKT_PREC_FP64, s);
    if (st != KKT_OK) return st;
    h->fp64_current = h->opts.precision == KKT_PREC_MIXED;
    h->factor_precision = h->opts.precision;
    h->repivots += 1;
    return KKT_OK;
}

// Validates a batch for kkt_refactor_batch(_graph): 1..kMaxBatch distinct bound handles of one
// analysis with the same precision and guard policy, and a value array for each.
kkt_status_t check_batch(const kkt_handle_t *hs, const double *const *dev_values, int32_t count) {
    if (!hs || !dev_values || count < 1 || count > kMaxBatch)
        return fail(hs && count > 0 ? hs[0] : nullptr, KKT_EINVAL, "need 1..8 handles and value arrays");
    for (int b = 0; b < count; ++b) {
        kkt_handle_t h = hs[b];
        if (!h || !dev_values[b]) return fail(hs[0], KKT_EINVAL, "null handle or value array in the batch");
        if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
        if (!h->bound) return fail(h, KKT_ESTATE, "no workspace bound");
        if (h->analysis_id != hs[0]->analysis_id || h->opts.precision != hs[0]->opts.precision ||
            h->opts.guard_policy != hs[0]->opts.guard_policy || h->device != hs[0]->device)
            return fail(hs[0], KKT_EINVAL,
                        "a batch needs handles of one analysis with the same precision, guard policy and device");
        for (int c = 0; c < b; ++c)
            if (hs[c] == h) return fail(hs[0], KKT_EINVAL, "a handle appears twice in the batch");
    }
    return KKT_OK;
}

// Graphs captured by kkt_refactor_batch_graph, one per (handles, their workspace bindings,
// precision); an entry is dropped when one of its handles is released.
struct BatchGraph {
    std::vector<kkt_handle_t> hs;
    std::vector<uint64_t> gens;
    int precision = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
constexpr size_t kMaxGraphs = 128;
std::mutex g_graph_mu;
std::vector<BatchGraph> g_graphs;

void drop_graphs_of(kkt_handle_t h) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size();) {
        if (std::find(g_graphs[i].hs.begin(), g_graphs[i].hs.end(), h) != g_graphs[i].hs.end()) {
            (void)hipGraphExecDestroy(g_graphs[i].exec);
            (void)hipGraphDestroy(g_graphs[i].graph);
            g_graphs.erase(g_graphs.begin() + i);
        } else {
            ++i;
        }
    }
}

// Device address of `scratch` on the current device, looked up once per device (each GPU
// holds its own copy of the array).  The host-side name `scratch` is not a device address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// x = Q U^-1 L^-1 P b with the current factors of precision T, the intermediate vectors and
// the tile counters in the static scratch at `base` (device address).
template <typename T>
hipError_t direct_solve_scratch(kkt_handle_t h, const double *b, double *x, unsigned char *base, hipStream_t s) {
    NoAllocHead *head = (NoAllocHead *)base;
    T *y = (T *)(base + kNoAllocHead);
    T *z = (T *)(base + kNoAllocHead + sizeof(double) * (size_t)kNoAllocMaxRows);
    k_fill_sentinel<T><<<h->grid_stream, kStreamBlock, 0, s>>>(h->an.n, y, z, &head->work_lower, &head->work_upper,
                                                                &head->hang);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_trsv<T>(h, true, b, nullptr, y, nullptr, nullptr, s, false, &head->work_lower, &head->hang);
    if (e != hipSuccess) return e;
    return launch_trsv<T>(h, false, nullptr, y, z, x, nullptr, s, false, &head->work_upper, &head->hang);
}

}  // namespace
}  // namespace kkt

static kkt_status_t solve_vorder(kkt_handle_t h, const double *dev_b, double tol, kkt_solve_info_t *info,
                                 hipStream_t s);

extern "C" {

void kkt_opts_default(kkt_opts_t *o) {
    if (!o) return;
    *o = kkt_opts_t{};  // every field not set below is 0 (tile_lds_kib, narrow_columns: automatic)
    o->ordering = KKT_ORDER_MD;
    o->nd_leaf = 64;
    o->pivot_tau = 1e-10;
    o->restart = 10;
    o->max_restarts = 20;
    o->delta_tol = 1e-14;
    o->nrbe_target = 1e-12;
    o->precision = KKT_PREC_FP64;
    o->guard_policy = KKT_GUARD_PERTURB;
    o->stop_mode = KKT_STOP_PAPER;
    o->mixed_fallback = 1;
    o->mixed_max_cycles = 3;
    o->ir_method = KKT_IR_FGMRES;
    o->richardson_max_it = 50;
    o->ratio_stop = 0.5;
    o->inner_tol = 1e-2;
    o->residual = KKT_RESID_FP64;
    o->repivot_cycles = 3;
    o->gram_schmidt = KKT_GS_CGS2;
    o->deterministic = 1;
}

kkt_status_t kkt_analyze(const kkt_opts_t *opts, int64_t n, const int64_t *rowptr, const int32_t *colidx,
                         const double *values_first, kkt_handle_t *out) {
    if (!out) return fail(nullptr, KKT_EINVAL, "null output handle");
    *out = nullptr;
    kkt_handle_t h = new (std::nothrow) kkt_handle_s();
    if (!h) return fail(nullptr, KKT_ENOMEM, "out of host memory");
    if (opts) h->opts = *opts;
    else kkt_opts_default(&h->opts);
    if (h->opts.restart < 1 || h->opts.restart > kRestartMax) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "restart must be in 1..64");
    }
    if (h->opts.gram_schmidt != KKT_GS_CGS2 && h->opts.gram_schmidt != KKT_GS_DCGS2) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "gram_schmidt must be KKT_GS_CGS2 or KKT_GS_DCGS2");
    }
    if (h->opts.residual != KKT_RESID_FP64 && h->opts.residual != KKT_RESID_DD) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "residual must be KKT_RESID_FP64 or KKT_RESID_DD");
    }
    if (h->opts.tile_lds_kib != 0 &&
        (h->opts.tile_lds_kib * 1024 < kTileLdsMin || h->opts.tile_lds_kib * 1024 > kTileLdsMax)) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "tile_lds_kib must be 0 or in 16..150");
    }
    if (h->opts.deterministic != 1) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "deterministic must be 1 (results are always bitwise repeatable)");
    }
    if (h->opts.narrow_columns < 0) {
        delete h;
        return fail(nullptr, KKT_EINVAL, "narrow_columns must be >= 0");
    }
    AnalysisOptions ao = analysis_options(h->opts, n);
    h->tile_lds = (size_t)ao.tile_lds;
    h->analysis_id = next_analysis_id();
    std::string msg;
    int rc = analyze(ao, n, rowptr, colidx, values_first, h->an, &msg);
    if (rc != AN_OK) {
        delete h;
        const kkt_status_t s = rc == AN_EINVAL ? KKT_EINVAL : rc == AN_ESINGULAR ? KKT_ESINGULAR : KKT_ENOMEM;
        return fail(nullptr, s, msg);
    }
    *out = h;
    return KKT_OK;
}

kkt_status_t kkt_get_analysis_info(kkt_handle_t h, kkt_analysis_info_t *info) {
    if (!h || !info) return fail(h, KKT_EINVAL, "null argument");
    const Analysis &a = h->an;
    info->n = a.n;
    info->nnz = a.nnz;
    info->nnz_l = a.nnz_l();
    info->nnz_u = a.nnz_u();
    info->offdiag_pivots = a.offdiag_pivots;
    info->levels_refactor = a.levels_refactor;
    info->levels_l = a.lsched.levels;
    info->levels_u = a.usched.levels;
    info->updates = a.updates();
    info->analysis_seconds = a.seconds;
    info->max_column = 0;
    for (int64_t j = 0; j < a.n; ++j) info->max_column = std::max(info->max_column, a.fp[j + 1] - a.fp[j]);
    info->tiles_l = a.lsched.tiles();
    info->tiles_u = a.usched.tiles();
    info->unstaged_l = (int64_t)std::count(a.lsched.tile_lds.begin(), a.lsched.tile_lds.end(), (uint8_t)0);
    info->unstaged_u = (int64_t)std::count(a.usched.tile_lds.begin(), a.usched.tile_lds.end(), (uint8_t)0);
    return KKT_OK;
}

kkt_status_t kkt_get_permutations(kkt_handle_t h, int32_t *prow, int32_t *q) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    if (prow) std::memcpy(prow, h->an.prow.data(), h->an.n * sizeof(int32_t));
    if (q) std::memcpy(q, h->an.q.data(), h->an.n * sizeof(int32_t));
    return KKT_OK;
}

kkt_status_t kkt_get_factor_pattern(kkt_handle_t h, int64_t *lp, int32_t *li, int64_t *up, int32_t *ui) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    const Analysis &a = h->an;
    if (lp) std::memcpy(lp, a.lp.data(), a.lp.size() * sizeof(int64_t));
    if (li) std::memcpy(li, a.li.data(), a.li.size() * sizeof(int32_t));
    if (up) std::memcpy(up, a.up.data(), a.up.size() * sizeof(int64_t));
    if (ui) std::memcpy(ui, a.ui.data(), a.ui.size() * sizeof(int32_t));
    return KKT_OK;
}

kkt_status_t kkt_get_analysis_values(kkt_handle_t h, double *lx, double *ux) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    if (lx) std::memcpy(lx, h->an.lx.data(), h->an.lx.size() * sizeof(double));
    if (ux) std::memcpy(ux, h->an.ux.data(), h->an.ux.size() * sizeof(double));
    return KKT_OK;
}

kkt_status_t kkt_workspace_size(kkt_handle_t h, int32_t batch, size_t *bytes) {
    if (!h || !bytes) return fail(h, KKT_EINVAL, "null argument");
    if (batch < 1) return fail(h, KKT_EINVAL, "batch must be at least 1");
    *bytes = plan(h).total * (size_t)batch;
    return KKT_OK;
}

kkt_status_t kkt_bind_workspace(kkt_handle_t h, void *dev_ptr, size_t bytes, void *stream) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    const Offsets o = plan(h);
    if (!dev_ptr || bytes < o.total) return fail(h, KKT_ENOMEM, "workspace too small");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(h, KKT_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    KKT_HIP(h, hipGetDevice(&h->device));
    h->bind_gen = next_analysis_id();
    if (!h->host_ctl) {
        KKT_HIP(h, hipHostMalloc((void **)&h->host_ctl, sizeof(ControlSummary),
                                 hipHostMallocMapped | hipHostMallocCoherent));
        KKT_HIP(h, hipHostGetDevicePointer((void **)&h->dev_ctl_sum, h->host_ctl, 0));
    }
    if (!h->host_rec) {
        KKT_HIP(h, hipHostMalloc((void **)&h->host_rec, sizeof(StepRecord) * (kRestartMax + 1),
                                 hipHostMallocMapped | hipHostMallocCoherent));
        KKT_HIP(h, hipHostGetDevicePointer((void **)&h->dev_rec, h->host_rec, 0));
    }
    for (int e = 0; e < 2; ++e)
        if (!h->step_ev[e]) KKT_HIP(h, hipEventCreateWithFlags(&h->step_ev[e], hipEventDisableTiming));
    char *b = (char *)dev_ptr;
    DevLayout &d = h->d;
    const Analysis &a = h->an;
    d.fp = (int64_t *)(b + o.fp);
    d.fi = (int32_t *)(b + o.fi);
    d.fdiag = (int32_t *)(b + o.fdiag);
    d.order = (int32_t *)(b + o.order);
    d.clev = (int32_t *)(b + o.clev);
    d.f2t = (int32_t *)(b + o.f2t);
    d.relptr = (int64_t *)(b + o.relptr);
    d.fsrc = (int64_t *)(b + o.fsrc);
    d.relpos = (int32_t *)(b + o.relpos);
    d.relsrc = (int32_t *)(b + o.relsrc);
    d.relslot = (int32_t *)(b + o.relslot);
    d.pc = (int64_t *)(b + o.pc);
    d.pu = (int64_t *)(b + o.pu);
    d.pnu = (int32_t *)(b + o.pnu);
    d.item = (int32_t *)(b + o.item);
    d.item_lane = (uint8_t *)(b + o.item_lane);
    d.krp = (int64_t *)(b + o.krp);
    d.kci = (int32_t *)(b + o.kci);
    d.l_rows = (int32_t *)(b + o.l_rows);
    d.l_seg = (int32_t *)(b + o.l_seg);
    d.l_tdesc = (int32_t *)(b + o.l_tdesc);
    d.l_src = (int32_t *)(b + o.l_src);
    d.l_src_k = (int32_t *)(b + o.l_src_k);
    d.l_ref = (int32_t *)(b + o.l_ref);
    d.l_esrc = (int32_t *)(b + o.l_esrc);
    d.l_rent = (int64_t *)(b + o.l_rent);
    d.l_sdof = (int32_t *)(b + o.l_sdof);
    d.l_slg = (int32_t *)(b + o.l_slg);
    d.u_rows = (int32_t *)(b + o.u_rows);
    d.u_seg = (int32_t *)(b + o.u_seg);
    d.u_tdesc = (int32_t *)(b + o.u_tdesc);
    d.u_q = (int32_t *)(b + o.u_q);
    d.u_q_k = (int32_t *)(b + o.u_q_k);
    d.u_ref = (int32_t *)(b + o.u_ref);
    d.u_esrc = (int32_t *)(b + o.u_esrc);
    d.u_rent = (int64_t *)(b + o.u_rent);
    d.u_sdof = (int32_t *)(b + o.u_sdof);
    d.u_slg = (int32_t *)(b + o.u_slg);
    d.prow = (int32_t *)(b + o.prow);
    d.q = (int32_t *)(b + o.q);
    d.vperm = (int32_t *)(b + o.vperm);
    d.prow_k = (int32_t *)(b + o.prow_k);
    d.q_k = (int32_t *)(b + o.q_k);
    d.ostart = (int64_t *)(b + o.ostart);
    d.fsrc32 = (int32_t *)(b + o.fsrc32);
    d.kval = (double *)(b + o.kval);
    d.F64 = (double *)(b + o.F64);
    d.T64 = (double *)(b + o.T64);
    d.F32 = (float *)(b + o.F32);
    d.T32 = (float *)(b + o.T32);
    d.Ld64 = (double *)(b + o.Ld64);
    d.Ld32 = (float *)(b + o.Ld32);
    d.V = (double *)(b + o.V);
    d.Z = (double *)(b + o.Z);
    d.w = (double *)(b + o.w);
    d.r = (double *)(b + o.r);
    d.y64 = (double *)(b + o.y64);
    d.z64 = (double *)(b + o.z64);
    d.y32 = (float *)(b + o.y32);
    d.z32 = (float *)(b + o.z32);
    d.dv = (double *)(b + o.dv);
    d.rr = (double *)(b + o.rr);
    d.xb = (double *)(b + o.xb);
    d.bi = (double *)(b + o.bi);
    d.xi = (double *)(b + o.xi);
    d.part = (double *)(b + o.part);
    d.ctl = (Control *)(b + o.ctl);
    KKT_HIP(h, up(b, o.fp, a.fp, s));
    KKT_HIP(h, up(b, o.fi, a.fi, s));
    KKT_HIP(h, up(b, o.fdiag, a.fdiag, s));
    KKT_HIP(h, up(b, o.order, a.col_order, s));
    KKT_HIP(h, up(b, o.clev, a.col_level, s));
    KKT_HIP(h, up(b, o.f2t, a.f2t, s));
    KKT_HIP(h, up(b, o.relptr, a.relptr, s));
    if (a.phys) {
        const std::vector<int32_t> f32(a.fsrc_k.begin(), a.fsrc_k.end());
        KKT_HIP(h, up(b, o.fsrc32, f32, s));
        KKT_HIP(h, hipStreamSynchronize(s));  // f32 is a local
    } else {
        KKT_HIP(h, up(b, o.fsrc, a.fsrc_k, s));
    }
    KKT_HIP(h, up(b, o.relpos, a.relpos, s));
    KKT_HIP(h, up(b, o.relsrc, a.relsrc, s));
    KKT_HIP(h, up(b, o.relslot, a.relslot, s));
    KKT_HIP(h, up(b, o.pc, a.pc, s));
    KKT_HIP(h, up(b, o.pu, a.pu, s));
    KKT_HIP(h, up(b, o.pnu, a.pnu, s));
    KKT_HIP(h, up(b, o.item, a.ref_item, s));
    KKT_HIP(h, up(b, o.item_lane, a.ref_item_lane, s));
    KKT_HIP(h, up(b, o.krp, a.krp, s));
    KKT_HIP(h, up(b, o.kci, a.kci, s));
    {
        std::vector<int64_t> ost(a.n);
        for (int64_t k = 0; k < a.n; ++k) ost[k] = a.rowptr[a.vperm[k]];
        KKT_HIP(h, up(b, o.ostart, ost, s));
        KKT_HIP(h, hipStreamSynchronize(s));  // ost is a local
    }
    KKT_HIP(h, up(b, o.vperm, a.vperm, s));
    KKT_HIP(h, up(b, o.prow_k, a.prow_k, s));
    KKT_HIP(h, up(b, o.q_k, a.q_k, s));
    KKT_HIP(h, up(b, o.l_rows, a.lsched.rows, s));
    KKT_HIP(h, up(b, o.l_seg, a.lsched.seg_row, s));
    // per-tile descriptors and the per-position right-hand-side sources / solution targets
    {
        const std::vector<int32_t> ld = tile_descriptors(a.lsched), ud = tile_descriptors(a.usched);
        std::vector<int32_t> ls(a.n), lsk(a.n), uq(a.n), uqk(a.n);
        for (int64_t p = 0; p < a.n; ++p) {
            ls[p] = a.prow[a.lsched.rows[p]];
            lsk[p] = a.prow_k[a.lsched.rows[p]];
            uq[p] = a.q[a.usched.rows[p]];
            uqk[p] = a.q_k[a.usched.rows[p]];
        }
        KKT_HIP(h, up(b, o.l_tdesc, ld, s));
        KKT_HIP(h, up(b, o.u_tdesc, ud, s));
        KKT_HIP(h, up(b, o.l_src, ls, s));
        KKT_HIP(h, up(b, o.l_src_k, lsk, s));
        KKT_HIP(h, up(b, o.u_q, uq, s));
        KKT_HIP(h, up(b, o.u_q_k, uqk, s));
        KKT_HIP(h, hipStreamSynchronize(s));  // the vectors are locals
    }
    KKT_HIP(h, up(b, o.l_ref, a.lsched.ent_ref, s));
    KKT_HIP(h, up(b, o.l_esrc, a.lsched.ext_src, s));
    KKT_HIP(h, up(b, o.l_rent, a.lsched.row_ent, s));
    KKT_HIP(h, up(b, o.l_sdof, a.lsched.seg_dofs, s));
    KKT_HIP(h, up(b, o.l_slg, a.lsched.seg_lg, s));
    KKT_HIP(h, up(b, o.u_rows, a.usched.rows, s));
    KKT_HIP(h, up(b, o.u_seg, a.usched.seg_row, s));
    KKT_HIP(h, up(b, o.u_ref, a.usched.ent_ref, s));
    KKT_HIP(h, up(b, o.u_esrc, a.usched.ext_src, s));
    KKT_HIP(h, up(b, o.u_rent, a.usched.row_ent, s));
    KKT_HIP(h, up(b, o.u_sdof, a.usched.seg_dofs, s));
    KKT_HIP(h, up(b, o.u_slg, a.usched.seg_lg, s));
    KKT_HIP(h, up(b, o.prow, a.prow, s));
    KKT_HIP(h, up(b, o.q, a.q, s));
    KKT_HIP(h, hipMemsetAsync(d.ctl, 0, sizeof(Control), s));
    // dense blocks of the solve layout hold explicit zeros that the refactorization never writes
    KKT_HIP(h, hipMemsetAsync(d.T64, 0, a.t_size * sizeof(double), s));
    KKT_HIP(h, hipMemsetAsync(d.T32, 0, a.t_size * sizeof(float), s));
    KKT_HIP(h, hipMemsetAsync(d.part, 0, (size_t)3 * kStreamGridMax * kPartStride * sizeof(double), s));
    KKT_HIP(h, hipStreamSynchronize(s));
    // at least one block per hand-out queue
    const bool flat = !h->an.relsrc.empty();
    // at most 3 blocks per compute unit: the flat variant fits 4, which measured slower (more
    // waiting columns in flight, 2M refactorization 0.98 against 1.02 ms)
    int cus = 0;
    KKT_HIP(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    const int cap = 3 * std::max(cus, 1);
    h->grid_refactor64 = std::max(kWorkQueues, std::min(cap, coop_grid(flat ? (const void *)k_refactor<double, true>
                                                                            : (const void *)k_refactor<double, false>,
                                                                       h->device)));
    h->grid_refactor32 = std::max(kWorkQueues, std::min(cap, coop_grid(flat ? (const void *)k_refactor<float, true>
                                                                            : (const void *)k_refactor<float, false>,
                                                                       h->device)));
    h->grid_trsv64 = std::min(std::min(coop_grid((const void *)k_trsv<double, true, true>, h->device, h->tile_lds),
                                       coop_grid((const void *)k_trsv<double, false, true>, h->device, h->tile_lds)),
                              std::min(coop_grid((const void *)k_trsv<double, true, false>, h->device, h->tile_lds),
                                       coop_grid((const void *)k_trsv<double, false, false>, h->device, h->tile_lds)));
    h->grid_trsv32 = std::min(std::min(coop_grid((const void *)k_trsv<float, true, true>, h->device, h->tile_lds),
                                       coop_grid((const void *)k_trsv<float, false, true>, h->device, h->tile_lds)),
                              std::min(coop_grid((const void *)k_trsv<float, true, false>, h->device, h->tile_lds),
                                       coop_grid((const void *)k_trsv<float, false, false>, h->device, h->tile_lds)));
    if (h->grid_refactor64 <= 0 || h->grid_refactor32 <= 0 || h->grid_trsv64 <= 0 || h->grid_trsv32 <= 0)
        return fail(h, KKT_EDEVICE, "occupancy query failed");
    h->grid_stream = stream_blocks(a.n);
    h->ws = b;
    h->ws_bytes = bytes;
    h->bound = true;
    h->have_factors = false;
    return KKT_OK;
}

kkt_status_t kkt_refactor(kkt_handle_t h, const double *dev_values, void *stream) {
    if (!h || !dev_values) return fail(h, KKT_EINVAL, "null argument");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    if (!h->bound) return fail(h, KKT_ESTATE, "no workspace bound");
    h->fp64_current = false;
    return refactor_impl(h, dev_values, h->opts.precision, (hipStream_t)stream);
}

kkt_status_t kkt_refactor_batch(const kkt_handle_t *hs, const double *const *dev_values, int32_t count,
                                void *stream) {
    const kkt_status_t st = check_batch(hs, dev_values, count);
    if (st != KKT_OK) return st;
    for (int b = 0; b < count; ++b) hs[b]->fp64_current = false;
    return refactor_batch_impl(hs, dev_values, count, hs[0]->opts.precision, (hipStream_t)stream);
}

kkt_status_t kkt_refactor_batch_graph(const kkt_handle_t *hs, const double *const *dev_values, int32_t count,
                                      void *stream) {
    kkt_status_t st = check_batch(hs, dev_values, count);
    if (st != KKT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the values go into each workspace's copy of K first (with ||K||_inf and their
    // finiteness); the graph refactors from there
    for (int b = 0; b < count; ++b) {
        const DevLayout &d = hs[b]->d;
        k_prep_values<<<1, 1, 0, s>>>(d.ctl);
        k_ingest_rows<<<ingest_grid(hs[b]->an.n), 256, 0, s>>>(hs[b]->an.n, d.ostart, d.krp, dev_values[b], d.kval,
                                                             d.ctl);
        KKT_HIP(hs[b], hipGetLastError());
    }
    const int precision = hs[0]->opts.precision;
    std::vector<uint64_t> gens(count);
    for (int b = 0; b < count; ++b) gens[b] = hs[b]->bind_gen;
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (const BatchGraph &g : g_graphs)
            if (g.precision == precision && g.gens == gens &&
                std::equal(g.hs.begin(), g.hs.end(), hs, hs + count) && (int)g.hs.size() == count)
                exec = g.exec;
    }
    if (!exec) {
        const std::vector<const double *> staged(count, nullptr);
        // Capture only records the launches, so it runs on a private stream (the caller's may be
        // the legacy default stream, which cannot capture); the graph is launched on the
        // caller's stream below.  No per-launch timing events inside a graph.
        hipStream_t cs = nullptr;
        KKT_HIP(hs[0], hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        const uint32_t mask = hs[0]->prof_mask;
        hs[0]->prof_mask = 0;
        hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        st = eb == hipSuccess ? refactor_batch_impl(hs, staged.data(), count, precision, cs) : KKT_OK;
        hipGraph_t graph = nullptr;
        const hipError_t ec = eb == hipSuccess ? hipStreamEndCapture(cs, &graph) : eb;
        hs[0]->prof_mask = mask;
        (void)hipStreamDestroy(cs);
        if (st != KKT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        KKT_HIP(hs[0], ec);
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            KKT_HIP(hs[0], ei);
        }
        BatchGraph g;
        g.hs.assign(hs, hs + count);
        g.gens = gens;
        g.precision = precision;
        g.graph = graph;
        g.exec = exec;
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (g_graphs.size() >= kMaxGraphs) {  // the oldest goes
            (void)hipGraphExecDestroy(g_graphs.front().exec);
            (void)hipGraphDestroy(g_graphs.front().graph);
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back(g);
    }
    KKT_HIP(hs[0], hipGraphLaunch(exec, s));
    for (int b = 0; b < count; ++b) {
        hs[b]->fp64_current = false;
        hs[b]->have_factors = true;
        hs[b]->factor_precision = precision;
        ++hs[b]->graph_launches;
    }
    return KKT_OK;
}

kkt_status_t kkt_graph_launches(kkt_handle_t h, int64_t *launches) {
    if (!h || !launches) return fail(h, KKT_EINVAL, "null argument");
    *launches = h->graph_launches;
    return KKT_OK;
}

kkt_status_t kkt_solve(kkt_handle_t h, const double *dev_b, double *dev_x, double tol, kkt_solve_info_t *info,
                       void *stream) {
    if (!h || !dev_b || !dev_x) return fail(h, KKT_EINVAL, "null argument");
    if (dev_b == dev_x) return fail(h, KKT_EINVAL, "b and x must be distinct");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    if (!h->bound || !h->have_factors) return fail(h, KKT_ESTATE, "refactor before solve");
    if (tol <= 0.0) tol = h->opts.delta_tol;
    hipStream_t s = (hipStream_t)stream;
    // the solve runs in the vector order: b in, then x out (the best iterate also when the
    // refinement misses the tolerance)
    const kkt_status_t st = solve_vorder(h, dev_b, tol, info, s);
    if (st == KKT_OK || st == KKT_ENOCONV) {
        k_vscatter<<<h->grid_stream, kStreamBlock, 0, s>>>(h->an.n, h->d.vperm, h->d.xi, dev_x);
        KKT_HIP(h, hipGetLastError());
    }
    return st;
}

}  // extern "C"

// kkt_solve in the vector order of the handle's analysis: b (the caller's, original order)
// is gathered into the workspace's b, the solution is left in its x.  A re-pivot re-lays out
// the workspace, so both are taken from the layout after it (and b gathered again).
static kkt_status_t solve_vorder(kkt_handle_t h, const double *dev_b, double tol, kkt_solve_info_t *info,
                                 hipStream_t s) {
    auto gather_b = [&]() -> kkt_status_t {
        k_vgather<<<h->grid_stream, kStreamBlock, 0, s>>>(h->an.n, h->d.vperm, dev_b, h->d.bi);
        KKT_HIP(h, hipGetLastError());
        return KKT_OK;
    };
    if (gather_b() != KKT_OK) return KKT_EDEVICE;
    const int cycles = h->opts.max_restarts + 1;
    if (h->factor_precision == KKT_PREC_MIXED && !h->fp64_current) {
        const int mixed_cycles = h->opts.mixed_fallback ? std::min(cycles, std::max(1, h->opts.mixed_max_cycles))
                                                        : cycles;
        kkt_status_t st = solve_impl<float>(h, h->d.bi, h->d.xi, tol, info, s, mixed_cycles);
        if (st != KKT_ENOCONV || !h->opts.mixed_fallback) return st;
        // FP64 fallback: refactor the values already in the workspace in FP64 (the FP32
        // factors stay valid); later solves of this system go straight to FP64
        st = refactor_impl(h, nullptr, KKT_PREC_FP64, s);
        if (st != KKT_OK) return st;
        h->factor_precision = KKT_PREC_MIXED;
        h->fp64_current = true;
    }
    kkt_status_t st;
    if (h->opts.ir_method == KKT_IR_RICHARDSON || h->opts.ir_method == KKT_IR_ERROR_FGMRES) {
        st = richardson_impl<double>(h, h->d.bi, h->d.xi, tol, info, s, h->opts.ir_method == KKT_IR_ERROR_FGMRES);
    } else {
        const bool rp = h->opts.repivot_cycles > 0;
        st = solve_impl<double>(h, h->d.bi, h->d.xi, tol, info, s,
                                rp ? std::min(cycles, h->opts.repivot_cycles) : cycles);
        if (st == KKT_ENOCONV && rp) {
            st = repivot_impl(h, s);
            if (st != KKT_OK) return st;
            if (gather_b() != KKT_OK) return KKT_EDEVICE;
            st = solve_impl<double>(h, h->d.bi, h->d.xi, tol, info, s, cycles);
            if (info) info->repivoted = 1;
        }
    }
    if (info && h->fp64_current) info->fallback = 1;
    return st;
}

extern "C" {

kkt_status_t kkt_direct_solve(kkt_handle_t h, const double *dev_b, double *dev_x, void *stream) {
    if (!h || !dev_b || !dev_x) return fail(h, KKT_EINVAL, "null argument");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    if (!h->bound || !h->have_factors) return fail(h, KKT_ESTATE, "refactor before solve");
    hipStream_t s = (hipStream_t)stream;
    if (h->factor_precision == KKT_PREC_MIXED) {
        rearm<float>(h, s);
        KKT_HIP(h, precond<float>(h, dev_b, dev_x, nullptr, s, false));
    } else {
        rearm<double>(h, s);
        KKT_HIP(h, precond<double>(h, dev_b, dev_x, nullptr, s, false));
    }
    return KKT_OK;
}

kkt_status_t kkt_direct_solve_noalloc(kkt_handle_t h, const double *dev_b, double *dev_x, void *stream) {
    if (!h || !dev_b || !dev_x) return fail(h, KKT_EINVAL, "null argument");
    if (h->an.n > kNoAllocMaxRows)
        return fail(h, KKT_EINVAL, "kkt_direct_solve_noalloc: n = " + std::to_string(h->an.n) +
                                       " exceeds its static scratch of " + std::to_string(kNoAllocMaxRows) + " rows");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    if (!h->bound || !h->have_factors) return fail(h, KKT_ESTATE, "refactor before solve");
    int dev = -1;
    KKT_HIP(h, hipGetDevice(&dev));
    if (dev != h->device) return fail(h, KKT_EINVAL, "the handle's device must be current");
    void *base = nullptr;
    KKT_HIP(h, scratch_address(dev, &base));
    hipStream_t s = (hipStream_t)stream;
    if (h->factor_precision == KKT_PREC_MIXED)
        KKT_HIP(h, direct_solve_scratch<float>(h, dev_b, dev_x, (unsigned char *)base, s));
    else
        KKT_HIP(h, direct_solve_scratch<double>(h, dev_b, dev_x, (unsigned char *)base, s));
    return KKT_OK;
}

kkt_status_t kkt_residual(kkt_handle_t h, const double *dev_b, const double *dev_x, double *dev_r, void *stream) {
    if (!h || !dev_b || !dev_x || !dev_r) return fail(h, KKT_EINVAL, "null argument");
    if (h->device_failed) return fail(h, KKT_EDEVICE, "handle unusable after a device error");
    if (!h->bound || !h->have_factors) return fail(h, KKT_ESTATE, "refactor before the residual");
    if (dev_r == dev_b || dev_r == dev_x) return fail(h, KKT_EINVAL, "dev_r must be distinct from dev_b and dev_x");
    hipStream_t s = (hipStream_t)stream;
    const KrylovArgs ka = kargs<double>(h);
    const int G = h->grid_stream;
    k_vgather<<<G, kStreamBlock, 0, s>>>(h->an.n, h->d.vperm, dev_b, h->d.bi);
    k_vgather<<<G, kStreamBlock, 0, s>>>(h->an.n, h->d.vperm, dev_x, h->d.xi);
    launch_resid(h, ka, h->d.bi, h->d.xi, h->d.r, s);
    k_vscatter<<<G, kStreamBlock, 0, s>>>(h->an.n, h->d.vperm, h->d.r, dev_r);
    KKT_HIP(h, hipGetLastError());
    return KKT_OK;
}

kkt_status_t kkt_get_factor_values(kkt_handle_t h, int32_t precision, double *lx, double *ux, void *stream) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    if (!h->bound || !h->have_factors) return fail(h, KKT_ESTATE, "no factors");
    hipStream_t s = (hipStream_t)stream;
    const Analysis &a = h->an;
    // the refactorization leaves its final values only in the solve layout, where f2t maps
    // every factor position
    const int64_t nt = a.t_size;
    std::vector<double> T(nt);
    if (precision == 1) {
        std::vector<float> T32(nt);
        KKT_HIP(h, hipMemcpyAsync(T32.data(), h->d.T32, nt * sizeof(float), hipMemcpyDeviceToHost, s));
        KKT_HIP(h, hipStreamSynchronize(s));
        for (int64_t t = 0; t < nt; ++t) T[t] = (double)T32[t];
    } else {
        KKT_HIP(h, hipMemcpyAsync(T.data(), h->d.T64, nt * sizeof(double), hipMemcpyDeviceToHost, s));
        KKT_HIP(h, hipStreamSynchronize(s));
    }
    if (lx)
        for (int64_t p = 0; p < a.nnz_l(); ++p) lx[p] = T[a.f2t[a.l2f[p]]];
    if (ux)
        for (int64_t p = 0; p < a.nnz_u(); ++p) ux[p] = T[a.f2t[a.u2f[p]]];
    return KKT_OK;
}

kkt_status_t kkt_set_profiling(kkt_handle_t h, int32_t on) {
    return kkt_set_profiling_mask(h, on ? (1u << KKT_K_CLASSES) - 1u : 0u);
}

kkt_status_t kkt_set_profiling_mask(kkt_handle_t h, uint32_t class_mask) {
    if (!h) return fail(h, KKT_EINVAL, "null handle");
    if (class_mask >> KKT_K_CLASSES) return fail(h, KKT_EINVAL, "class mask has bits beyond KKT_K_CLASSES");
    h->prof_mask = class_mask;
    h->times = kkt_kernel_times_t{};
    return KKT_OK;
}

kkt_status_t kkt_get_kernel_times(kkt_handle_t h, kkt_kernel_times_t *t, void *stream) {
    if (!h || !t) return fail(h, KKT_EINVAL, "null argument");
    if (!h->ev_pending.empty()) {
        KKT_HIP(h, hipStreamSynchronize((hipStream_t)stream));
        prof_collect(h);
    }
    *t = h->times;
    return KKT_OK;
}

kkt_status_t kkt_clone(kkt_handle_t src, kkt_handle_t *out) {
    if (!src || !out) return fail(src, KKT_EINVAL, "null argument");
    *out = nullptr;
    kkt_handle_t h = new (std::nothrow) kkt_handle_s();
    if (!h) return fail(src, KKT_ENOMEM, "out of host memory");
    try {
        h->opts = src->opts;
        h->an = src->an;
        h->tile_lds = src->tile_lds;
        h->analysis_id = src->analysis_id;
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(src, KKT_ENOMEM, "out of host memory");
    }
    *out = h;
    return KKT_OK;
}

kkt_status_t kkt_release(kkt_handle_t h) {
    if (!h) return KKT_OK;
    drop_graphs_of(h);
    for (auto &r : h->ev_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->host_ctl) (void)hipHostFree(h->host_ctl);
    if (h->host_rec) (void)hipHostFree(h->host_rec);
    for (auto e : h->step_ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return KKT_OK;
}

const char *kkt_last_error(kkt_handle_t h) {
    if (h) return h->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
