// Device-side data structures shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kkt {

constexpr int kRestartMax = 64;        // largest supported FGMRES restart length
constexpr int kStreamBlock = 256;      // threads per block of the streaming kernels
constexpr int kStreamGridMax = 1024;   // blocks of the streaming kernels (partial-sum rows)
constexpr int kCoopBlock = 256;        // threads per block of the refactorization
constexpr int kTileThreads = 256;      // threads per block of the triangular solves
constexpr int kTileRows = 2048;        // rows of a multi-level solve tile (values in LDS)
constexpr int kTileLds = 32768;        // default LDS bytes of a staged solve tile
constexpr int kTileLdsMin = 16 * 1024;  // smallest and largest tile budgets (gfx950: 160 KiB of LDS
constexpr int kTileLdsMax = 150 * 1024; // per compute unit, the rest for the kernel's own arrays)
// Wavefronts the refactorization keeps resident on an MI355X: 3 blocks of 4 per compute unit,
// 256 compute units.
constexpr int kResidentRefactorWaves = 3 * 4 * 256;
constexpr int kRefactorLds = 1024;     // factor entries staged in LDS per wavefront
constexpr int kMaxBatch = 8;           // systems of one pattern refactored by one launch
constexpr int kWorkQueues = 8;         // refactorization hand-out queues (one per XCD of MI355X: a
                                       // block's queue is its index mod 8, the XCD it runs on)
// Spin limit of one dependency wait (iterations of a short sleep, a few seconds in all);
// exceeding it marks Control::hang and lets every wave run to completion.
constexpr unsigned int kSpinLimit = 1u << 22;

// Scalars shared between kernels of one refactor/solve (device memory).
struct Control {
    unsigned long long knorm_bits;  // max_i sum_j |K_ij| as the bits of a non-negative double
    unsigned int nonfinite;         // a non-finite matrix value was ingested
    unsigned int guard_fail;        // a guarded pivot under the FAIL policy
    unsigned long long nguard;      // guarded (perturbed) pivots
    unsigned int counter;           // arrival counter of the "last block reduces" pattern
    int stop;                       // current FGMRES cycle has ended
    int jdone;                      // Arnoldi steps completed in the current cycle
    int breakdown;                  // happy breakdown in the current cycle
    int nonfinite_b;                // non-finite right-hand side
    unsigned int hang;              // a dependency wait exceeded its spin limit
    double beta;                    // ||rho|| at the start of the cycle
    double inner_tol;               // stop when the estimated residual <= inner_tol
    double est;                     // estimated residual |g_{j+1}|
    double wnorm_in;                // ||K z_j|| before orthogonalization
    double hn;                      // ||w|| after CGS2
    double rnorm2, xnorm2, bnorm2;  // sums of squares from the residual kernel
    double rinf, xinf;              // max |rho_i|, max |x_i| from the residual kernel
    double h1[kRestartMax + 1];     // first CGS pass coefficients
    double h2[kRestartMax + 1];     // second CGS pass coefficients
    double g[kRestartMax + 1];      // g[j]: right-hand side entry j before rotation j is applied
    double gr[kRestartMax];         // gr[j]: entry j after rotation j (the least-squares rhs); kept
                                    // apart from g so that no block of the normalization kernel
                                    // reads a value block 0 rewrites in the same launch
    double cs[kRestartMax], sn[kRestartMax];
    double y[kRestartMax];          // least-squares solution of the cycle
    double H[(kRestartMax + 1) * kRestartMax];  // rotated Hessenberg (upper triangular), column-major
    double Hbar[(kRestartMax + 1) * kRestartMax];  // DCGS2: final columns before rotation
    double hp[2][kRestartMax + 1];  // DCGS2: one-pass column j in hp[j & 1] (read by step j + 1)
    // Refactorization hand-out: kWorkQueues counters, one per 256-byte line; queue q hands out
    // items q, q + kWorkQueues, ... to the blocks b with b % kWorkQueues == q.
    unsigned int work_refactor[kWorkQueues * 64];
    unsigned int work_lower;        // next task index to hand out (L solve)
    unsigned int work_upper;        // next task index to hand out (U solve)
};

// What the host needs after each Arnoldi step, written by the normalization kernel into
// pinned host memory (one record per step of the cycle).
struct StepRecord {
    int stop;
    unsigned int hang;
    int jdone;
    int pad;
    double est;
    unsigned long long token;  // written last (release): identifies the step the record is for
};

// Host-visible summary copied back once per cycle.
struct ControlSummary {
    unsigned long long knorm_bits;
    unsigned int nonfinite;
    unsigned int guard_fail;
    unsigned long long nguard;
    unsigned int counter;
    int stop, jdone, breakdown, nonfinite_b;
    unsigned int hang;
    double beta, inner_tol, est, wnorm_in, hn, rnorm2, xnorm2, bnorm2, rinf, xinf;
};

}  // namespace kkt
