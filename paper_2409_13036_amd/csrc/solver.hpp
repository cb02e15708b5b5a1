// Host drivers of the PCG solves (solver.cpp).
#pragma once

#include <vector>

#include "internal.hpp"

namespace rafem {

struct SolveOpts {
    double tol = 1e-10;
    int maxit = 20000;
    int precision = RAFEM_FP64;
    double inner_tol = 1e-4;
    int max_outer = 30;
    int poll_every = 0;
    int restart_inner = 0;
};

SolveOpts resolve_opts(const rafem_solve_opts* o, double default_tol);

// hints (optional, in/out): iteration counts of the previous solve of the same kind (FP64:
// one count; MIXED: one per inner solve), the first-chunk guesses of this solve; replaced
// by this solve's counts.

// FP64 Jacobi-PCG on A from x (in/out).  dinv may be NULL for a CSR matrix (then it is
// computed from A's diagonal).  Fills info, returns its status.
rafem_status pcg64(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv,
                   const double* b, double* x, const SolveOpts& o, rafem_solve_info* info,
                   hipStream_t s, std::vector<int>* hints);

// FP32 inner PCG (on A.v32) inside FP64 iterative refinement (on A.v).  dinv/dinv32 may be
// NULL for a CSR matrix.
rafem_status pcg_mixed(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv,
                       const float* dinv32, const double* b, double* x, const SolveOpts& o,
                       rafem_solve_info* info, hipStream_t s, std::vector<int>* hints);

// A whole solve of one system enqueued with fixed budgets and no host synchronisation
// (rafem_solve_enqueue): FP64, `iterations` PCG iterations; mixed, `refinements` refinements
// of at most `iterations` inner iterations each and the residual check of the last; the
// report written to info_d.  A is a CSR matrix (D^-1 computed from its diagonal).
void solve_enqueue(rafem_mesh m, const Mat& A, const Samples& smp, const double* b, double* x,
                   const SolveOpts& o, int iterations, int refinements,
                   rafem_device_info* info_d, hipStream_t s);

// Pick the SELL slab shape of the FP64 and FP32 SpMV by timing them on A (sets m->tuned).
void autotune_spmv(rafem_mesh m, const Mat& A, hipStream_t s);

// Device-driven form of a solve: everything is enqueued at once, the iteration budget of
// each (inner) solve taken from `hints` (the previous solve of the same kind), and the
// solver states are copied into log slots from m->dd_used on after each of them; no host
// synchronisation.  A mixed solve enqueues one refinement more than the hints hold, which
// only checks the last one when the count was right.  The record says where the logs are.
struct DdRecord {
    int slot0 = 0;
    int rounds = 0;          // logged slots (1 for FP64)
    int mixed = 0;
    std::vector<int> budget; // iterations enqueued per slot
};
// Whether device-driven enqueueing is possible for this solve (hints present, fit the log).
bool dd_ready(rafem_mesh m, const SolveOpts& o, const std::vector<int>* hints);
DdRecord dd_enqueue(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv,
                    const float* dinv32, const double* b, double* x, const SolveOpts& o,
                    const std::vector<int>& hints, hipStream_t s);
// After the caller's poll of the log slots into m->dd_log_host: true if the enqueued solve
// did exactly what the host-driven solve does (every inner solve finished within its budget,
// every sample converged, no refinement the host would have judged stagnant); then fills
// info, the per-sample counters and hints.  h_out receives the log slot holding the final
// states (main FP64 states at [0, S) and true residuals at [2S, 3S); mixed: refinement
// states at [S, 2S)).
bool dd_finish(rafem_mesh m, const DdRecord& r, const SolveOpts& o, rafem_solve_info* info,
               std::vector<int>* hints, const PcgState** h_out);

}  // namespace rafem
