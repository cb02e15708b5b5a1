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

// SELL layout with slabs of 64 rows (one wavefront, one row per lane).
struct HostSell {
    int64_t nslabs = 0;
    std::vector<int32_t> sptr;  // [nslabs + 1] element offset of each slab
    std::vector<int32_t> scol;  // [sptr[nslabs]] column ids, slab-major, entry-major within slab
    std::vector<int32_t> rlen;  // [n] entries of each row that may be nonzero (no padding)
    std::vector<int16_t> sdel;  // column - row offsets of the slabs with sofs = -1, or empty
    std::vector<int32_t> sofs;  // [nslabs] start of a shared-offset slab's list in soff; else
                                // -1: per-slot columns, 16-bit in sdel if it is not empty;
                                // -2: per-slot 32-bit columns (offsets beyond 16 bits)
    std::vector<int32_t> soff;  // offset lists of the shared-offset slabs, slab by slab
};
// row_off: sample boundaries ({0, n} for one mesh); no slab offset crosses them.
HostSell build_sell(const HostStructure& S, int64_t n, const std::vector<int64_t>& row_off);

// Node -> element incidences as CSR by node: list[k] = e npe + a (conn[e][a] = node), elements
// ascending.
void node_elements(int64_t n, int64_t E, int npe, const int32_t* conn, std::vector<int32_t>& ptr,
                   std::vector<int32_t>& list);
// Throws Error on bad input.
void check_conn(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn);
HostStructure build_structure(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn);
constexpr int kColourWords = 4;  // colour masks of 4 x 64 bits: at most 256 colours
int colour_elements(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn,
                    int32_t* colour);
// Reverse Cuthill-McKee order of the node graph: order[k] = node placed at position k.
std::vector<int32_t> rcm_order(int64_t n, const HostStructure& S);
// Stable sort of order[] by node degree within consecutive windows of positions.
void degree_sort(int64_t n, const HostStructure& S, int64_t window, int32_t* order);
// Minimum Jacobian determinant over the quadrature points of every element (hex: 2x2x2
// Gauss points; tet: the constant determinant).  Throws E_MESH if any is <= 0.
// Returns true when every element is affine (hex: a parallelepiped; tets always are).
bool check_geometry(int64_t n_elems, int npe, const int32_t* conn, const double* xyz);

// ---------------------------------------------------------------------------
// Device-side solver state.  One instance per concurrent reduction chain.
// Written only by the "last block" of a kernel or by k_state_init.
// ---------------------------------------------------------------------------
struct PcgState {
    double rzs[2];   // (r, D^-1 r) of the current residual, slot = iteration parity
    double pq;       // (p, A p) of the last iteration (diagnostics)
    double beta;
    double rr;       // ||r||^2 of the current residual
    double bb;       // ||b||^2
    double tol;      // relative tolerance
    double tol2;     // tol^2 * bb: stop when rr <= tol2
    double scale;    // mixed refinement: 1 / ||r_outer||
    double rr_first; // ||r||^2 at the start of this solve
    double scale_prev; // mixed refinement: the scale of the previous refinement
    int32_t iters;
    int32_t maxit;
    int32_t done;
    int32_t status;
    int32_t bad_diag;
    int32_t pad;
};
static_assert(sizeof(PcgState) % 8 == 0, "PcgState layout");
static_assert(sizeof(PcgState) <= 128, "PcgState size (3 states per sample fill 384 bytes at most)");

// Launch geometry of the row kernels.
struct SpmvConfig {
    int lanes;            // CSR kernels: lanes per row (2, 4, 8 or 16)
    int rows_per_block;   // CSR kernels: multiple of 256 / lanes
    int slabs_per_block;  // SELL kernels: 64-row slabs per 256-thread workgroup (multiple of 4)
    int stream = 0;       // SELL kernels: 1 = matrix values read with nontemporal loads...
    int resident = 0;     // ...past this many value slots (the prefix with ordinary loads)
    int min_blocks = 1;   // SELL kernels: launch bound in workgroups per CU, 1 or kSellMinBlocks
};
constexpr int kSellMinBlocks = 6;

SpmvConfig choose_spmv_config(int64_t n, int64_t nnz);
int blocks_for(int64_t n, int rows_per_block);
constexpr int kVecRowsPerBlock = 1024;  // vector kernels: 256 threads x 4 rows

// A sparse matrix as the solver kernels see it: CSR, or SELL with 64-row slabs.
struct Mat {
    int32_t n = 0;
    int sell = 0;
    const int32_t* rp = nullptr;    // CSR row pointers [n + 1]
    const int32_t* ci = nullptr;    // CSR column ids [nnz]
    int32_t nslabs = 0;
    const int32_t* sptr = nullptr;  // SELL slab offsets [nslabs + 1]
    const int32_t* scol = nullptr;  // SELL column ids [sptr[nslabs]]
    const int16_t* sdel = nullptr;  // SELL column - row offsets (slabs with sofs -1), or NULL
    int wide = 0;                   // SELL: some slabs have sofs -2 (32-bit columns) as well
    const int32_t* sofs = nullptr;  // SELL [nslabs]: start of a slab's shared offsets, or -1 / -2
                                    // (per-slot 16-bit / 32-bit columns, as in HostSell)
    const int32_t* soff = nullptr;  // SELL shared offset lists
    const double* v = nullptr;      // values in the layout's order
    const float* v32 = nullptr;     // FP32 values in the layout's order (mixed precision)
};

// Where the entries of a row live, for the element-wise kernels (assembly, lifting).
struct Layout {
    int sell = 0;
    const int32_t* rp = nullptr;    // CSR
    const int32_t* sptr = nullptr;  // SELL
    const int32_t* rlen = nullptr;  // SELL
    const int32_t* cols = nullptr;  // column ids in the layout's order
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All asynchronous on `s`.
// ---------------------------------------------------------------------------
// A batch of independent systems: sample s owns rows [row_off[s], row_off[s+1]) (device
// array); interior offsets are multiples of kRowAlign so no workgroup spans two samples.
constexpr int kRowAlign = 1024;
struct Samples {
    int S;
    const int32_t* row_off;
    const int32_t* tab = nullptr;  // [rows / kRowAlign] sample of each aligned block, or NULL
    int max_rows = 0;              // rows of the largest sample (0: unknown)
};

// Grid of a row kernel: blocks and rows per block (to locate a sample's partial slots).
struct GridInfo {
    int nb = 0;
    int rpb = 1;
};

// Solver states are arrays of S (one per sample).  itb points at the device iteration
// counter of the running loop (set to 0 by launch_state_init when given).
void launch_state_init(PcgState* st, int S, double tol, int maxit, int* itb, hipStream_t s);
void launch_advance(int* itb, int k, hipStream_t s);
// dinv = 1 / diag(A) (CSR matrices, one system); a missing or non-positive diagonal marks
// st->bad_diag.
void launch_diag_inv(const Mat& A, double* dinv, float* dinv32, PcgState* st, hipStream_t s);
// r = b - A x; z = p = D^-1 r (z into the residual buffer); per-sample r.z, r.r, b.b into
// st (FP64 PCG start).
void launch_pcg_start(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                      const double* dinv, double* r, double* p, double* partials,
                      PcgState* st, const Samples& smp, hipStream_t s);
// One PCG iteration is three kernels.  None of them finalises a reduction itself: each
// writes per-block partial sums, and every block of the next kernel adds its sample's
// partials in a fixed order (kernel boundaries make them visible), so no fences or
// atomics are needed and all blocks of a sample see bit-identical scalars.  The
// iteration index is *itb + j; scalars carried between iterations live in slots chosen
// by its parity, so no kernel reads a slot it also writes.
//   spmv_dot:  q = A p; partial p.q per block into pq_part.
//   update:    pq = sum(pq_part); alpha = rz[it&1] / pq (breakdown if pq <= 0);
//              x += alpha p; z -= alpha D^-1 q (z = D^-1 r); partials of r.z and r.r
//              (r = z / D^-1) into rz_part.
//   pupdate:   rz', rr = sum(rz_part); stop on convergence / limit / breakdown, else
//              beta = rz' / rz[it&1]; p = z + beta p; rz[(it+1)&1] = rz'.
// All three skip the samples whose st->done is set.
// ev0 / ev1 (optional): events stamped at the kernel's own start and end
GridInfo launch_spmv_dot64(const Mat& A, const SpmvConfig& c, const double* p, double* q,
                           double* pq_part, PcgState* st, const Samples& smp, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
GridInfo launch_spmv_dot32(const Mat& A, const SpmvConfig& c, const float* p, float* q,
                           double* pq_part, PcgState* st, const Samples& smp, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// sums (optional, >= 3 S doubles): where a sample's totals are pre-summed by one block per
// sample when its partial slots are many (large meshes), so that the vector kernels' blocks
// do not each read them all; the totals are bitwise the same either way.
int launch_update64(int n, double* x, double* r, const double* p, const double* q,
                    const double* dinv, const double* pq_part, const GridInfo& gpq,
                    double* rz_part, const int* itb, int j, PcgState* st, const Samples& smp,
                    double* sums, hipStream_t s);
int launch_update32(int n, float* x, float* r, const float* p, const float* q, const float* dinv,
                    const double* pq_part, const GridInfo& gpq, double* rz_part, const int* itb,
                    int j, PcgState* st, const Samples& smp, double* sums, hipStream_t s);
void launch_pupdate64(int n, double* p, const double* z, const double* rz_part, int nb_rz,
                      const int* itb, int j, PcgState* st, const Samples& smp, double* sums,
                      hipStream_t s);
void launch_pupdate32(int n, float* p, const float* z, const double* rz_part, int nb_rz,
                      const int* itb, int j, PcgState* st, const Samples& smp, double* sums,
                      hipStream_t s);
// Plain y = A x (no state).
void launch_spmv64(const Mat& A, const SpmvConfig& c, const double* x, double* y, hipStream_t s);
void launch_spmv32(const Mat& A, const SpmvConfig& c, const float* x, float* y, hipStream_t s);
// Residual r = b - A x with ||r||^2 and ||b||^2 into st[s].rr, st[s].bb.  outer_mode (mixed
// refinement): skips finished samples, tol2 = tol^2 bb, done when rr <= tol2, else
// scale = 1/||r|| and one more refinement is counted.
void launch_residual64(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                       double* r, double* partials, PcgState* st, const Samples& smp,
                       int outer_mode, hipStream_t s);
// Mixed inner start: r32 = scale * r64; d32 = 0; rz, rr into the inner state.  A fresh
// start (cont = 0) sets p32 = D^-1 r32.  A continuation (cont = 1: a reliable update of the
// inner recurrence, after the previous inner solve reached its tolerance and x was
// refined) keeps the search direction: p32 = D^-1 r32 + beta p32 with the beta of the
// recurrence's next step, the new residual standing in for the recursive one and both
// brought to the new scale.
void launch_inner_start(int n, const double* r64, const PcgState* outer, float* r32, float* d32,
                        float* p32, const float* dinv32, double inner_tol, int maxit,
                        double* partials, PcgState* inner, const Samples& smp, int cont,
                        hipStream_t s);
// x64 += d32 / scale (samples whose refinement is not finished).
void launch_refine_update(int n, double* x, const float* d32, const PcgState* outer,
                          const Samples& smp, hipStream_t s);
// The device-side report of rafem_solve_enqueue (one sample): cleared; inner iterations
// added after each refinement; completed from the final state and the true residual
// (chk: rr, bb of b - A x).
void launch_info_begin(rafem_device_info* info, hipStream_t s);
void launch_info_add_inner(const PcgState* inner, rafem_device_info* info, hipStream_t s);
void launch_info_finish(const PcgState* st, const PcgState* chk, int mixed,
                        rafem_device_info* info, hipStream_t s);

// Assembly.
void launch_fill(double* v, int64_t n, double value, hipStream_t s);
void launch_fill32(float* v, int64_t n, float value, hipStream_t s);
void launch_scatter_dirichlet(const int32_t* dir_ids, const double* dir_vals, int64_t nD,
                              double* gnode, hipStream_t s);
void launch_set_dirichlet(const int32_t* dir_ids, const double* gnode, int64_t nD, double* x,
                          hipStream_t s);
// affine: every hex is a parallelepiped (closed-form element integrals); e2s: optional
// value position of every (element, a, b) in L (else searched).
void launch_assemble_colour(int npe, int affine, const int32_t* elems, int count,
                            const int32_t* conn, const double* xyz, const Layout& L,
                            const int32_t* e2s, const double* mass, const double* stiff,
                            double* vals, hipStream_t s);
void launch_slot_map(int64_t E, int npe, const int32_t* conn, const Layout& L, int32_t* e2s,
                     hipStream_t s);
// Row-wise assembly on the SELL layout (slabs at most kRowAsmMaxW wide): one wavefront per
// slab, one lane per row, the row's values summed over the node's incident elements in
// LDS, then lifted (as launch_lift), copied to FP32 and written once.  The incidences of
// slab b sit lane-interleaved at [isptr[b], isptr[b+1]): slot isptr[b] + k WAVE + l holds
// e npe + a of the k-th incident element of row 64 b + l (or -1), and byte c of r2j at the
// same slot the entry index within the row of column conn[e][c].
constexpr int kRowAsmMaxW = 64;
// Doubles per element of the geometric constants (parallelepiped hex, tet).
constexpr int kGeoHex = 8, kGeoTet = 16;
struct RowAsm {
    int n = 0, nslabs = 0, width = 0;  // width: widest slab (entries per row)
    const int32_t *sptr = nullptr, *scol = nullptr;
    const int32_t *isptr = nullptr, *n2e = nullptr;
    const uint64_t* r2j = nullptr;
    const uint64_t* dmask = nullptr;  // per row: bit j set when entry j is in a Dirichlet column
    const uint8_t* jdiag = nullptr;   // per row: index of the diagonal entry (255: none)
    const int32_t* conn = nullptr;
    const double* xyz = nullptr;
    const double* geo = nullptr;  // geometric constants (tets and parallelepiped hexes)
    const double *mass = nullptr, *stiff = nullptr;
    const uint8_t* isD = nullptr;
    const double* gnode = nullptr;
    int do_lift = 0;
    double* vals = nullptr;
    float* vals32 = nullptr;
    double *lift = nullptr, *dinv = nullptr;
    float* dinv32 = nullptr;
};
void launch_row_slots(int64_t total, int npe, const int32_t* n2e, const int32_t* conn,
                      const int32_t* e2s, const int32_t* sptr, uint64_t* r2j, hipStream_t s);
void launch_elem_geo(int64_t E, int npe, const int32_t* conn, const double* xyz, double* geo,
                     hipStream_t s);
void launch_assemble_rows(int npe, int affine, const RowAsm& a, hipStream_t s);
// Bioheat right-hand side with the row-wise assembly's incidences: every element's terms
// into erhs[e npe + a] (one launch over all elements; parallelepiped hexes from geo when
// given), then per row their sum, lifted into b as launch_finish_rhs does.
void launch_bioheat_rhs_rows(int npe, int affine, int64_t E, const int32_t* conn,
                             const double* xyz, const double* geo, const double* T, const double* V,
                             const double* sigma, const double* perf, double rho_c_dt, double T_a,
                             int with_joule, double* erhs, int n, const int32_t* isptr,
                             const int32_t* n2e, const double* lift, const uint8_t* isD,
                             double* b, hipStream_t s);
// Lifting with per-node Dirichlet mask/values; writes lifted vals, vals32, lift, dinv, dinv32.
void launch_lift(int n, const Layout& L, double* vals, float* vals32, const uint8_t* isD,
                 const double* gnode, double* lift, double* dinv, float* dinv32, int do_lift,
                 hipStream_t s);
void launch_cast32(const double* v, float* v32, int64_t n, hipStream_t s);
// coef[e] = c0 + perf[e]
void launch_coef(const double* perf, double c0, double* coef, int64_t E, hipStream_t s);
void launch_sigma(int npe, int64_t E, const int32_t* conn, const double* T, const double* sigma0,
                  double alpha, double T_ref, double* sigma, hipStream_t s);
void launch_bioheat_rhs_colour(int npe, int affine, const int32_t* elems, int count,
                               const int32_t* conn, const double* xyz, const double* T,
                               const double* V, const double* sigma, const double* perf,
                               double rho_c_dt, double T_a, int with_joule, double* rhs,
                               hipStream_t s);
// Reverse step of the coupled time step (adjoint.hip).
void launch_vjp_params(int npe, int affine, int64_t E, const int32_t* conn, const double* xyz,
                       const double* mu, const double* Tn, double T_a, double* grad_k,
                       double* grad_w, hipStream_t s);
void launch_vjp_joule_colour(int npe, int affine, const int32_t* elems, int count,
                             const int32_t* conn, const double* xyz, const double* V,
                             const double* mu, const double* sigma, double* nubar, double* sbar1,
                             hipStream_t s);
void launch_vjp_sigma(int npe, int affine, int64_t E, const int32_t* conn, const double* xyz,
                      const double* nu, const double* V, const double* sbar1,
                      const double* sigma0, double alpha, double* dsig, hipStream_t s);
void launch_vjp_lambda_colour(int npe, int affine, const int32_t* elems, int count,
                              const int32_t* conn, const double* xyz, const double* mu,
                              const double* dsig, double rho_c_dt, double* lam, hipStream_t s);
void launch_loss(int64_t n, const int32_t* ids, const double* target, const double* T,
                 double scale, double* grad, double* partials, double* loss, hipStream_t s);
// b = isD ? lift : rhs + lift
// out = a + c (a - b) (b may be NULL: out = a); the predictor's linear extrapolation.
void launch_extrapolate(int n, const double* a, const double* b, double c, double* out,
                        hipStream_t s);
// Polynomial predictor out = sum_k w[k] x[k], k < terms (3 to 5).
void launch_extrapolate_poly(int n, int terms, const double* const* x, const double* w,
                             double* out, hipStream_t s);
// norm2[0] = sum (x - y)^2, norm2[1] = sum x^2, deterministically (partials: >= n/256 + 1).
void launch_change_norm(int n, const double* x, const double* y, double* partials,
                        double* norm2, hipStream_t s);
void launch_finish_rhs(int n, const double* rhs, const double* lift, const uint8_t* isD,
                       double* b, hipStream_t s);


// Helpers of the C ABI layer (abi.cpp): device memory owned by the handle, and the
// handle's SELL and CSR layouts.
void* mesh_alloc(rafem_mesh m, size_t bytes);
Layout mesh_sell_layout(rafem_mesh m);
Layout mesh_csr_layout(rafem_mesh m);

// ---------------------------------------------------------------------------
// Monolithic (T, V) corrector: Jacobian assembly, block SpMV and GMRES(m) (gmres.hip).
// ---------------------------------------------------------------------------
constexpr int kGmMaxM = RAFEM_GMRES_MAX_M;

// Device state of one GMRES solve (written by the single-thread kernels only).
struct GmState {
    double tol, bnorm, beta, est, relres_true;
    int32_t iters, cycles, jdone, cyc_done, solved, status, maxit, m;
};

// The basis (vector i of the interleaved (T, V) pairs at V + i ldv; double2 or, fp32,
// float2 elements), the per-block partial sums [rows][nb] and the state.
struct GmVec {
    int n;
    void* V;
    int64_t ldv;
    double* part;
    GmState* st;
    int fp32 = 0;
};

// Hessenberg matrix (column-major, leading dimension ldh), rotations, rotated right-hand
// side, least-squares solution, and the per-step residual estimates (hist, may be NULL).
struct GmSmall {
    double* H;
    int ldh;
    double *cs, *sn, *g, *y;
    double* hist;
    int hist_cap;
};

struct BsellArgs {
    int n = 0, nslabs = 0;
    const int32_t* sptr = nullptr;
    const int32_t* scol = nullptr;
    const int16_t* sdel = nullptr;
    const int32_t* sofs = nullptr;
    const int32_t* soff = nullptr;
    const void* vals = nullptr;     // (TT, TV, VT, VV) per slot: double4, or float4 if fp32
    const void* x = nullptr;        // double2 / float2 per node
    void* y = nullptr;
    const GmState* st = nullptr;    // skip when the solve (or, arnoldi: the cycle) is over
    int arnoldi = 0;
    int fp32 = 0;
};

// One colour of the Jacobian / residual assembly.  Value c (0..3 = TT, TV, VT, VV) of
// slot k goes to vals[k * slot_mul + c * plane_stride]; R[2i], R[2i+1] += rsign * (R_T, R_V).
struct JacArgs {
    const int32_t* elems = nullptr;
    int count = 0;
    const int32_t* conn = nullptr;
    const double* xyz = nullptr;
    Layout L;
    const int32_t* e2s = nullptr;
    const uint8_t* isD = nullptr;
    const double *Tn = nullptr, *T = nullptr, *V = nullptr;
    const double *k_e = nullptr, *perf = nullptr, *sigma0 = nullptr;
    double rho_c_dt = 0.0, T_a = 0.0, alpha = 0.0, T_ref = 0.0;
    double* vals = nullptr;
    int64_t plane_stride = 1;
    int slot_mul = 4;
    double* R = nullptr;
    double rsign = 1.0;
};

void launch_jac_assemble_colour(int npe, int affine, const JacArgs& a, hipStream_t s);
void launch_jac_dirichlet(const int32_t* dir_ids, int64_t nD, const Layout& L, double* vals,
                          int slot_mul, int64_t plane_stride, hipStream_t s);
// binv[4i..4i+3] = inverse of node i's diagonal block (vals4: SELL slots of double4).
void launch_block_inv(int n, const Layout& L, const double* vals4, double* binv, hipStream_t s);
void launch_bsell(const BsellArgs& a, hipStream_t s);
int gm_blocks(int n);  // workgroups (= partial slots) of the per-node GMRES kernels
void launch_gm_init(GmState* st, double tol, int maxit, int m, hipStream_t s);
// Vector arguments (w, z, r, binv) have the basis' precision (fp32: float2 / float4), except
// in launch_gm_xupdate (delta, binv: FP64) and launch_gm_resid (b, w, r: FP64).
// launch_gm_dots / launch_gm_orth return the number of partial slots they wrote (the nb
// of the launch_gm_sum that reduces them).
int launch_gm_dots(const GmVec& a, int k, const void* w, hipStream_t s);
void launch_gm_sum(const double* part, int nb, int rows, double* out, const GmState* st,
                   hipStream_t s);
int launch_gm_orth(const GmVec& a, int k, const double* h1, void* w, hipStream_t s);
void launch_gm_next(const GmVec& a, int k, const double* h2, const void* w, const void* binv,
                    void* z, hipStream_t s);
void launch_gm_givens(const GmSmall& sm, int j, const double* h1, const double* h2, GmState* st,
                      hipStream_t s);
void launch_gm_solve_y(const GmSmall& sm, const GmState* st, hipStream_t s);
void launch_gm_xupdate(const GmVec& a, const double* y, const double* binv, double* delta,
                       hipStream_t s);
void launch_gm_resid(const GmVec& a, const double* b, const double* w, double* r, hipStream_t s);
void launch_gm_restart(const double* part, int nb, const GmSmall& sm, GmState* st, int first,
                       hipStream_t s);
void launch_gm_v0(const GmVec& a, const double* r, const void* binv, void* z, hipStream_t s);
// T += delta.T, V += delta.V; norm2 = (||delta_T||^2, ||T||^2) (part: >= 2 gm_blocks(n)).
void launch_newton_apply(int n, const double* delta, double* T, double* V, double* part,
                         double* norm2, hipStream_t s);

// ---------------------------------------------------------------------------
// Mesh handle.
// ---------------------------------------------------------------------------
}  // namespace rafem

// The solves of a step and of its reverse, each with its own chunk hints.
constexpr int kSolvePotential = 0, kSolveBioheat = 1, kSolveAdjointBioheat = 2,
              kSolveAdjointPotential = 3;

struct rafem_mesh_s {
    int64_t n = 0, E = 0, nnz = 0, nD = 0;
    int npe = 0, n_colours = 0;
    int device = 0;
    std::vector<int32_t> colour_off;  // host [n_colours + 1]
    rafem::SpmvConfig spmv{4, 512, 8};    // FP64 kernels
    rafem::SpmvConfig spmv32{4, 512, 8};  // FP32 kernels
    bool tuned = false;                   // slab shapes picked by the autotuner
    bool tuned_from_cache = false;        // ... taken from its on-disk cache
    bool use_graphs = false;              // iteration chunks captured as HIP graphs
    bool graphs_small = false;            // ...in rafem_step's solves of a small single mesh
    hipStream_t gstream = nullptr;        // capture stream
    struct GraphEntry {
        int kind;
        const void* key[4];
        int len;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;

    // structure and geometry
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    int64_t sell_nnz = 0;     // padded SELL storage (values per matrix of the step path)
    int32_t nslabs = 0;
    int32_t* sptr = nullptr;  // SELL slab offsets
    int32_t* scol = nullptr;  // SELL column ids
    int32_t* rlen = nullptr;  // SELL row lengths
    int32_t* e2s = nullptr;   // value position in the SELL layout of every (element, a, b)
    // row-wise assembly (every slab at most kRowAsmMaxW wide): node -> element incidences and
    // the entry index of every (incidence, b) within its row
    bool row_asm = false;
    int max_w = 0;  // widest slab (entries per row)
    int32_t *isptr = nullptr, *n2e = nullptr;
    uint64_t* r2j = nullptr;
    uint64_t* dmask = nullptr;
    uint8_t* jdiag = nullptr;
    double* geo = nullptr;    // per-element geometric constants of the row-wise assembly
    double* erhs = nullptr;   // per-incidence terms of the bioheat right-hand side
    int affine = 0;           // every hex is a parallelepiped
    int16_t* sdel = nullptr;  // SELL column - row offsets (NULL when no slab is within int16 reach)
    int32_t* sofs = nullptr;  // [nslabs] start of a shared-offset slab's list in soff, or -1 / -2
    int32_t* soff = nullptr;  // offset lists of the shared-offset slabs
    int64_t shared_slabs = 0;
    int64_t int32_slabs = 0;  // slabs that read 32-bit columns
    int64_t index_bytes = 0;  // column data (offsets, slab pointers) one SpMV reads
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
    double bioheat_dt = 0.0;       // time step the bioheat matrix was assembled for
    // predictor-corrector step: T^n and V^n (restored on rejection), the current iterate,
    // and the two sums of the change norm
    double *pc_Tn = nullptr, *pc_Vn = nullptr, *pc_Tk = nullptr, *pc_norm = nullptr;
    // extrapolated starting points of rafem_step (phys->extrapolate): the states at the start
    // of the last calls: slot xg_cur receives the next; the kept earlier states T^{n-k}
    // (k = 1 .. xg_kept) sit in slot (xg_cur - k) mod kXgSlots, xg_h[k-1] being the time step
    // that led from T^{n-k} to T^{n-k+1}
    static constexpr int kXgSlots = 5;
    double* xg_T[kXgSlots] = {};
    double* xg_V[kXgSlots] = {};
    int xg_cur = 0;
    int xg_kept = 0;
    double xg_h[kXgSlots - 1] = {};
    bool potential_ready = false;  // a step has assembled the potential matrix
    double *adj_mu = nullptr, *adj_nu = nullptr, *adj_sbar = nullptr, *adj_dsig = nullptr;
    bool adj_kept = false, adj_kept_nu = false;  // mu (nu) of the last reverse step kept
    // iteration counts of the previous solve of each kind and precision (first-chunk guesses)
    std::vector<int> hints[4][2];
    std::vector<int> hints_prev[4][2];  // the counts of the solve before (device-driven budgets)
    // how the solves of the current step start (rafem_step: the predictor's order q, or -1
    // from the previous state; -2 other entry points), and how the solves behind hints and
    // hints_prev started: device-driven budgets come only from solves that started alike
    int step_q = -2;
    int hints_q[4][2] = {{-3, -3}, {-3, -3}, {-3, -3}, {-3, -3}};
    int hints_prev_q[4][2] = {{-3, -3}, {-3, -3}, {-3, -3}, {-3, -3}};

    // monolithic corrector (allocated on first use): Jacobian slots as double4 in the SELL
    // layout, -R, block-Jacobi inverses, the Newton update, GMRES vectors and basis
    double *mono_vals = nullptr, *mono_rhs = nullptr, *mono_binv = nullptr, *mono_delta = nullptr;
    float *mono_vals32 = nullptr, *mono_binv32 = nullptr;  // FP32 copies (mixed GMRES)
    double *gm_w = nullptr, *gm_z = nullptr, *gm_r = nullptr, *gm_part = nullptr;
    double* gm_small = nullptr;        // H, cs, sn, g, y, h1, h2
    double* gm_V = nullptr;            // basis, (gm_cap + 1) vectors (freed on growth)
    int gm_cap = 0;
    rafem::GmState* gm_st = nullptr;
    rafem::GmState* gm_st_host = nullptr;  // pinned
    // solver workspace
    double *r = nullptr, *p = nullptr, *q = nullptr, *dinv = nullptr, *r64 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr, *dinv32 = nullptr;
    double* partials = nullptr;   // once-per-solve reductions
    double* part_pq = nullptr;    // per-iteration partials of p.Ap
    double* part_rz = nullptr;    // per-iteration partials of r.z and r.r
    double* part_sum = nullptr;   // [3 S] pre-summed totals of the two (large meshes)
    int max_sample_rows = 0;      // rows of the largest sample
    rafem::PcgState* st = nullptr;      // device [3 S]: main/inner, outer, check per sample
    rafem::PcgState* st_host = nullptr; // pinned host [3 S]
    int32_t* itb = nullptr;             // device iteration counters [2]: FP64 loop, inner loop
    int S = 1;                          // samples in the batch
    std::vector<int64_t> node_off;      // host [S + 1] first node of each sample (padded layout)
    std::vector<int64_t> elem_off;      // host [S + 1]
    std::vector<int64_t> dir_off;       // host [S + 1]
    int32_t* row_off = nullptr;         // device [S + 1]
    int32_t* row_tab = nullptr;         // device [n / kRowAlign] sample of each 1024-row block
    int32_t* row_off_one = nullptr;     // device {0, n}: the whole mesh as one system
    std::vector<rafem_step_info> sample_info;  // per-sample info of the last step
    std::vector<int> mixed_iters;   // per sample: inner (+ FP64 fallback) iterations of the last mixed solve
    std::vector<char> mixed_fell;   // per sample: 1 if that solve was finished by FP64 PCG

    // region timing (rafem_regions_*): events at region boundaries within a step, the
    // region of the interval each one opens, and the accumulated milliseconds per region
    bool reg_on = false;
    std::vector<hipEvent_t> reg_ev;
    std::vector<int> reg_kind;
    double reg_ms[3] = {0.0, 0.0, 0.0};
    int64_t reg_steps = 0;

    // measurement of the SpMV kernels (rafem_profile_*)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;   // 2 per launch, kProfCap launches
    double prof_sum_us[2] = {0.0, 0.0};  // [0] FP64 kernel, [1] FP32 kernel
    int64_t prof_cnt[2] = {0, 0};

    // device-driven solves (rafem_mesh_set_device_driven; off by default): each solve
    // of a step is enqueued whole, its iteration budgets taken from the previous solves'
    // counts, and the solver states are logged after every (inner) solve; one poll at its
    // end checks the logs, and a solve whose budgets fell short is redone from its saved
    // starting point host-driven
    bool dd_on = false;
    double dd_scale = 1.05;               // budget = ceil(count * dd_scale) + kDdSlack
    rafem::PcgState* dd_log = nullptr;       // device [kDdSlots][3 S]
    rafem::PcgState* dd_log_host = nullptr;  // pinned mirror
    double* dd_x0 = nullptr;              // the solve's starting point
    int dd_used = 0;                      // log slots used by the current solve
    int64_t dd_solves = 0, dd_redone = 0; // device-driven solves accepted / redone

    std::vector<void*> allocations;
};

namespace rafem {
constexpr int kProfCap = 2048;
constexpr int64_t kGraphSmallRows = 262144;     // single meshes up to this size replay graphs
constexpr int kDdMaxRounds = 15;                  // refinements enqueued per mixed solve, at most
constexpr int kDdSlots = kDdMaxRounds + 1;        // log slots of one solve
constexpr int kDdSlack = 3;                       // iterations added to every budget
}
