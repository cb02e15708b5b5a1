// Host drivers of the monolithic (T, V) corrector (mono.cpp).
#pragma once

#include "internal.hpp"

namespace rafem {

struct GmresOpts {
    int m = 30;
    int maxit = 20000;
    double tol = 1e-10;
    int precision = RAFEM_FP64;
};

GmresOpts resolve_gmres(const rafem_gmres_opts* o);

// Workspace of the monolithic corrector for restart length mvec (allocated once, the
// basis grown when a longer restart is asked for; fp32: also the FP32 copies of J and of
// the block inverses, which mono_assemble then keeps current).
void mono_ensure(rafem_mesh m, int mvec, bool fp32);

// J (SELL slots, m->mono_vals), -R (m->mono_rhs) and the block-Jacobi inverses at (T, V).
void mono_assemble(rafem_mesh m, const rafem_phys* phys, const double* k_e, const double* perf,
                   const double* sigma0, const double* Tn, const double* T, const double* V,
                   hipStream_t s);

// J as four planes in CSR order and R, into caller buffers.
void mono_export(rafem_mesh m, const rafem_phys* phys, const double* k_e, const double* perf,
                 const double* sigma0, const double* Tn, const double* T, const double* V,
                 double* planes, double* R, hipStream_t s);

// Restarted right-preconditioned GMRES(o.m) on the assembled J from x = 0; returns the
// status (also in info).
rafem_status gmres_solve(rafem_mesh m, const double* b, double* x, const GmresOpts& o,
                         double* hist, int hist_cap, rafem_gmres_info* info, hipStream_t s);

}  // namespace rafem
