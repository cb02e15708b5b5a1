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

// Pick the SELL slab shape of the FP64 and FP32 SpMV by timing them on A (sets m->tuned).
void autotune_spmv(rafem_mesh m, const Mat& A, hipStream_t s);

}  // namespace rafem
