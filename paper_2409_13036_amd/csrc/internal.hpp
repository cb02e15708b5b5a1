// Internal declarations of the rafem library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rafem.h"

namespace rafem {

// ---------------------------------------------------------------------------
// Error handling: thread-local message, status codes from rafem.h.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

struct Error {
    rafem_status code;
    std::string msg;
};

#define RAFEM_HIP(call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::rafem::Error{RAFEM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// ---------------------------------------------------------------------------
// Host-side mesh analysis (structure.cpp).
// ---------------------------------------------------------------------------
struct HostStructure {
    std::vector<int32_t> row_ptr;
    std::vector<int32_t> col_idx;
};

// Throws Error on bad input.
void check_conn(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn);
HostStructure build_structure(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn);
int colour_elements(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn,
                    int32_t* colour);
// Minimum Jacobian determinant over the quadrature points of every element (hex: 2x2x2
// Gauss points; tet: the constant determinant).  Throws E_MESH if any is <= 0.
void check_geometry(int64_t n_elems, int npe, const int32_t* conn, const double* xyz);

// ---------------------------------------------------------------------------
// Device-side solver state.  One instance per concurrent reduction chain.
// Written only by the "last block" of a kernel or by k_state_init.
// ---------------------------------------------------------------------------
struct PcgState {
    double rz;       // (r, D^-1 r) of the current residual
    double pq;       // (p, A p)
    double alpha;
    double beta;
    double rr;       // ||r||^2 of the current residual
    double bb;       // ||b||^2
    double tol;      // relative tolerance
    double tol2;     // tol^2 * bb: stop when rr <= tol2
    double scale;    // mixed refinement: 1 / ||r_outer||
    double rr_first; // ||r||^2 at the start of this solve
    int32_t iters;
    int32_t maxit;
    int32_t done;
    int32_t status;
    int32_t bad_diag;
    uint32_t ticket;  // arrival counter of the last-block reductions; 0 between kernels
};
static_assert(sizeof(PcgState) % 8 == 0, "PcgState layout");

// Launch geometry of the row kernels.
struct SpmvConfig {
    int lanes;           // lanes per row: 2, 4 or 8
    int rows_per_block;  // multiple of 256 / lanes
};

SpmvConfig choose_spmv_config(int64_t n, int64_t nnz);
int blocks_for(int64_t n, int rows_per_block);
constexpr int kVecRowsPerBlock = 1024;  // vector kernels: 256 threads x 4 rows

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All asynchronous on `s`.
// ---------------------------------------------------------------------------
struct Csr64 {
    const int32_t* rp;
    const int32_t* ci;
    const double* v;
    int32_t n;
};
struct Csr32 {
    const int32_t* rp;
    const int32_t* ci;
    const float* v;
    int32_t n;
};

void launch_state_init(PcgState* st, double tol, int maxit, hipStream_t s);
void launch_diag_inv(const Csr64& A, double* dinv, float* dinv32, PcgState* st, hipStream_t s);
// r = b - A x; p = D^-1 r; reduction of rz, rr, bb into st (FP64 PCG start).
void launch_pcg_start(const Csr64& A, const SpmvConfig& c, const double* b, const double* x,
                      const double* dinv, double* r, double* p, double* partials,
                      PcgState* st, hipStream_t s);
// q = A p; reduction of p.q into st, alpha = rz / pq.  Early exit when st->done.
void launch_spmv_dot64(const Csr64& A, const SpmvConfig& c, const double* p, double* q,
                       double* partials, PcgState* st, hipStream_t s);
void launch_spmv_dot32(const Csr32& A, const SpmvConfig& c, const float* p, float* q,
                       double* partials, PcgState* st, hipStream_t s);
// x += alpha p; r -= alpha q; rz, rr reductions; convergence test; beta.
void launch_update64(int n, double* x, double* r, const double* p, const double* q,
                     const double* dinv, double* partials, PcgState* st, hipStream_t s);
void launch_update32(int n, float* x, float* r, const float* p, const float* q,
                     const float* dinv, double* partials, PcgState* st, hipStream_t s);
// p = D^-1 r + beta p
void launch_pupdate64(int n, double* p, const double* r, const double* dinv, PcgState* st,
                      hipStream_t s);
void launch_pupdate32(int n, float* p, const float* r, const float* dinv, PcgState* st,
                      hipStream_t s);
// Plain y = A x (no state).
void launch_spmv64(const Csr64& A, const SpmvConfig& c, const double* x, double* y, hipStream_t s);
void launch_spmv32(const Csr32& A, const SpmvConfig& c, const float* x, float* y, hipStream_t s);
// Residual r = b - A x with ||r||^2 and ||b||^2 into st->rr, st->bb (no early exit).
// Mixed outer test: done when rr <= tol2 (tol2 = tol^2 bb set here), scale = 1/||r||.
void launch_residual64(const Csr64& A, const SpmvConfig& c, const double* b, const double* x,
                       double* r, double* partials, PcgState* st, int outer_mode, hipStream_t s);
// Mixed inner start: r32 = scale * r64; d32 = 0; p32 = D^-1 r32; rz, rr into inner state.
void launch_inner_start(int n, const double* r64, const PcgState* outer, float* r32, float* d32,
                        float* p32, const float* dinv32, double inner_tol, int maxit,
                        double* partials, PcgState* inner, hipStream_t s);
// x64 += d32 / scale (unless the outer state is done).
void launch_refine_update(int n, double* x, const float* d32, const PcgState* outer,
                          hipStream_t s);

// Assembly.
void launch_fill(double* v, int64_t n, double value, hipStream_t s);
void launch_scatter_dirichlet(const int32_t* dir_ids, const double* dir_vals, int64_t nD,
                              double* gnode, hipStream_t s);
void launch_set_dirichlet(const int32_t* dir_ids, const double* gnode, int64_t nD, double* x,
                          hipStream_t s);
void launch_assemble_colour(int npe, const int32_t* elems, int count, const int32_t* conn,
                            const double* xyz, const int32_t* rp, const int32_t* ci,
                            const double* mass, const double* stiff, double* vals,
                            hipStream_t s);
// Lifting with per-node Dirichlet mask/values; writes lifted vals, vals32, lift, dinv, dinv32.
void launch_lift(int n, const int32_t* rp, const int32_t* ci, double* vals, float* vals32,
                 const uint8_t* isD, const double* gnode, double* lift, double* dinv,
                 float* dinv32, int do_lift, hipStream_t s);
void launch_cast32(const double* v, float* v32, int64_t n, hipStream_t s);
// coef[e] = c0 + perf[e]
void launch_coef(const double* perf, double c0, double* coef, int64_t E, hipStream_t s);
void launch_sigma(int npe, int64_t E, const int32_t* conn, const double* T, const double* sigma0,
                  double alpha, double T_ref, double* sigma, hipStream_t s);
void launch_bioheat_rhs_colour(int npe, const int32_t* elems, int count, const int32_t* conn,
                               const double* xyz, const double* T, const double* V,
                               const double* sigma, const double* perf, double rho_c_dt,
                               double T_a, int with_joule, double* rhs, hipStream_t s);
// b = isD ? lift : rhs + lift
void launch_finish_rhs(int n, const double* rhs, const double* lift, const uint8_t* isD,
                       double* b, hipStream_t s);

// ---------------------------------------------------------------------------
// Mesh handle.
// ---------------------------------------------------------------------------
}  // namespace rafem

struct rafem_mesh_s {
    int64_t n = 0, E = 0, nnz = 0, nD = 0;
    int npe = 0, n_colours = 0;
    int device = 0;
    std::vector<int32_t> colour_off;  // host [n_colours + 1]
    rafem::SpmvConfig spmv{4, 512};

    // structure and geometry
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    int32_t* conn = nullptr;
    double* xyz = nullptr;
    int32_t* colour_elems = nullptr;
    int32_t* dir_ids = nullptr;
    uint8_t* isD = nullptr;

    // step buffers
    double *gV = nullptr, *gT = nullptr, *sigma = nullptr;
    double *valsV = nullptr, *liftV = nullptr, *dinvV = nullptr;
    double *valsT = nullptr, *liftT = nullptr, *dinvT = nullptr;
    float *valsV32 = nullptr, *valsT32 = nullptr, *dinvV32 = nullptr, *dinvT32 = nullptr;
    double *rhs = nullptr, *bT = nullptr, *gtmp = nullptr, *coefT = nullptr;
    bool bioheat_ready = false;
    int hint_V = 0, hint_T = 0;  // iterations of the previous FP64 solves, first-chunk guess

    // solver workspace
    double *r = nullptr, *p = nullptr, *q = nullptr, *dinv = nullptr, *r64 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr, *dinv32 = nullptr;
    double* partials = nullptr;
    rafem::PcgState* st = nullptr;      // device [3]: main/inner, outer, check
    rafem::PcgState* st_host = nullptr; // pinned host [3]

    // measurement of the SpMV kernels (rafem_profile_*)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;   // 2 per launch, kProfCap launches
    double prof_sum_us[2] = {0.0, 0.0};  // [0] FP64 kernel, [1] FP32 kernel
    int64_t prof_cnt[2] = {0, 0};

    std::vector<void*> allocations;
};

namespace rafem {
constexpr int kProfCap = 2048;
}
