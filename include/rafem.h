/*
 * rafem.h -- C ABI of the MI355X (gfx950) library for the per-time-step sparse
 * solves of a radiofrequency-ablation finite-element model.
 *
 * The operations follow the paper's problem statement:
 *   - each time step assembles the element equations of a tetrahedral (here
 *     also hexahedral) mesh into one global sparse matrix and solves A x = b
 *     (Sec. II-A, Fig. 1; Sec. II-B);
 *   - the global matrix is stored in CSR (Sec. III-A) and its sparsity
 *     structure does not change between steps, so it is analysed once per mesh
 *     and reused (Sec. III-B);
 *   - the solution stays in device memory between assembly and solve
 *     (Sec. III-A).
 * Each step is split into two symmetric positive-definite solves: the
 * quasi-static potential with temperature-dependent conductivity, then the
 * backward-Euler Pennes bioheat equation; both are solved with
 * Jacobi-preconditioned conjugate gradients (the paper names CG for SPD
 * systems and preconditioning in Sec. II-B).
 *
 * Conventions (all entry points):
 *   - Pointers ending in _h are host memory, pointers ending in _d are device
 *     memory on the current HIP device.  All _d buffers belong to the caller and
 *     must stay alive until the stream work that uses them has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it in stream order.  The solve entry points poll a few
 *     device scalars on that stream and return only when the solve has finished.
 *   - Opaque handles (rafem_mesh) and their workspaces belong to the library:
 *     they are allocated in rafem_mesh_create and freed by rafem_mesh_destroy.
 *     No other entry point allocates device memory, except the measurement call
 *     rafem_spmv_timing (its own temporary copies).
 *   - Argument and mesh errors are detected on the host before anything is
 *     enqueued; on such an error nothing is enqueued and the outputs are
 *     untouched.  Numerical failures (no convergence, breakdown) are reported in
 *     the info structs and by the return value; outputs then hold the last
 *     iterate.  No C++ exception crosses this boundary and the library never
 *     aborts the process.
 *   - A handle may be used by one host thread at a time.
 *   - Integer index arrays are int32, zero-based.  Node ids index [0, n_nodes).
 */
#ifndef RAFEM_H
#define RAFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Raised whenever a declaration below changes (a struct's layout, a signature). */
#define RAFEM_ABI_VERSION 3

typedef int32_t rafem_status;
#define RAFEM_OK            0  /* success */
#define RAFEM_E_ARG         1  /* bad argument: null pointer, size, option value */
#define RAFEM_E_MESH        2  /* bad mesh: node id out of range, element with detJ <= 0 */
#define RAFEM_E_NOCONV      3  /* iteration limit reached; outputs hold the last iterate */
#define RAFEM_E_BREAKDOWN   4  /* p.Ap <= 0 or a non-finite scalar: matrix not SPD or corrupt input */
#define RAFEM_E_HIP         5  /* a HIP runtime call failed (message from rafem_last_error) */
#define RAFEM_E_NOMEM       6  /* device or pinned host allocation failed */
#define RAFEM_E_STATE       7  /* call out of order (e.g. reuse requested before a first assembly) */

/* Message of the last failed call on this host thread; valid until the next call on it. */
const char* rafem_last_error(void);

/* RAFEM_ABI_VERSION of the loaded library. */
int32_t rafem_abi_version(void);

/* ---------------------------------------------------------------------------
 * Host-only mesh analysis (no GPU needed).  Sec. III-B: the matrix structure is
 * the same at every step, so it is computed once per mesh.
 * ------------------------------------------------------------------------- */

/* CSR pattern of the node graph of a mesh: entry (i, j) exists iff nodes i and j
 * share an element; every node's row holds its diagonal; columns ascending.
 * The pattern does not depend on boundary conditions.
 *   conn_h     [n_elems * npe] host, element-major node ids; npe is 8 (hex) or 4 (tet)
 *   nnz_out    receives the number of entries
 *   row_ptr_h  [n_nodes + 1] host output, or NULL to query nnz only
 *   col_idx_h  [nnz] host output, or NULL to query nnz only
 * Errors: E_ARG (sizes, null conn), E_MESH (node id outside [0, n_nodes), nnz > INT32_MAX). */
rafem_status rafem_csr_structure(int64_t n_nodes, int64_t n_elems, int32_t npe,
                                 const int32_t* conn_h, int64_t* nnz_out,
                                 int32_t* row_ptr_h, int32_t* col_idx_h);

/* Element colouring used for race-free assembly: elements of one colour share no
 * node, so their contributions to the global matrix can be added concurrently
 * without atomics.  Greedy first-fit in element order (at most 256 colours).
 *   colour_h       [n_elems] host output, colour of each element
 *   n_colours_out  receives the number of colours
 * Errors: E_ARG, E_MESH (node id out of range; more than 256 colours needed). */
rafem_status rafem_colour_elements(int64_t n_nodes, int64_t n_elems, int32_t npe,
                                   const int32_t* conn_h, int32_t* colour_h,
                                   int32_t* n_colours_out);

/* Reverse Cuthill-McKee ordering of the node graph (nodes adjacent when they share an
 * element), one of the reorderings of a sparse solver's analysis step (Sec. II-B): it
 * keeps the columns of each row, and so the x entries a slab of rows reads, close to the
 * row.  Per connected component, in order of its smallest node id: the pseudo-peripheral
 * start node of George and Liu (least degree, ties by smallest id), breadth-first search
 * taking unvisited neighbours by increasing degree (ties by smallest id); the
 * concatenated order reversed.  Host-only; deterministic.
 *   order_h  [n_nodes] host output: order_h[k] = the node placed at position k
 * Renumber a mesh by it (new id of node order_h[k] is k) before rafem_mesh_create.
 * Errors: E_ARG, E_MESH (node id out of range, repeated node in an element). */
rafem_status rafem_rcm_order(int64_t n_nodes, int64_t n_elems, int32_t npe,
                             const int32_t* conn_h, int32_t* order_h);

/* Within consecutive windows of `window` positions of a node order (e.g. the RCM order),
 * sort the nodes by increasing degree, ties kept in their order (host-only).  The rows of
 * each 64-row slab of the solver's layout then have nearly equal lengths, so little of the
 * slab is padding; the columns stay within about one window of the RCM bandwidth.
 *   order_h  [n_nodes] host, in: a permutation of the nodes; out: the sorted one
 * Errors: E_ARG (window < 1, order not a permutation), E_MESH as for rafem_rcm_order. */
rafem_status rafem_degree_sort(int64_t n_nodes, int64_t n_elems, int32_t npe,
                               const int32_t* conn_h, int64_t window, int32_t* order_h);

/* ---------------------------------------------------------------------------
 * Mesh handle: structure, colouring, geometry and all device workspaces.
 * ------------------------------------------------------------------------- */
typedef struct rafem_mesh_s* rafem_mesh;

typedef struct {
    int64_t n_nodes;
    int64_t n_elems;
    int64_t nnz;
    int64_t n_dirichlet;
    int32_t nodes_per_elem;
    int32_t n_colours;
    int32_t n_samples;
    int32_t slabs_per_block;     /* SELL shape of the FP64 SpMV (autotuned at the first step,
                                    with the choice of streamed value loads below) */
    int32_t slabs_per_block32;   /* SELL shape of the FP32 SpMV */
    int32_t int16_columns;       /* 1 if the SpMV reads 16-bit column offsets (on some slabs) */
    int64_t slabs;               /* 64-row slabs of the SpMV layout */
    int64_t shared_offset_slabs; /* slabs whose rows share one column-offset list */
    int32_t row_assembly;        /* 1: step matrices and right-hand side assembled row by row
                                    (every row has at most 64 entries), 0: colour by colour */
    int32_t max_row_entries;     /* entries of the longest row of the slab layout */
    int64_t value_slots;         /* stored values per matrix in the slab layout (padding included) */
    int64_t index_bytes;         /* column data one product reads: slab pointers, the shared
                                    offset lists, 16- or 32-bit per-slot column offsets */
    int32_t device_driven;       /* 1 if rafem_step's solves run device-driven (see
                                    rafem_mesh_set_device_driven) */
    int32_t tuned_from_cache;    /* 1 if the slab shapes came from the autotuner's on-disk cache
                                    (RAFEM_TUNE_CACHE, else ~/.cache/rafem/spmv_tune.txt) */
    int64_t device_driven_solves;/* solves of rafem_step completed device-driven */
    int64_t device_driven_redone;/* device-driven solves redone host-driven (a budget fell short) */
    int64_t int32_column_slabs;  /* slabs without a shared offset list whose columns lie beyond
                                    16-bit reach of their rows: they read 32-bit columns, the
                                    other such slabs 16-bit offsets */
    int32_t streamed_values;     /* 1 if the FP64 SpMV reads its values with nontemporal loads
                                    past a prefix (autotuned: matrices beyond the Infinity Cache) */
    int32_t streamed_values32;   /* the same for the FP32 SpMV */
    int64_t resident_slots;      /* that prefix: value slots read with ordinary loads (FP64) */
    int64_t resident_slots32;    /* the same for the FP32 SpMV */
    int32_t launch_bound;        /* resident workgroups per CU the FP64 SpMV kernel is compiled
                                    for: 1 (the compiler's register budget) or 6 (registers
                                    capped so that 6 fit); autotuned, the same bits either way */
    int32_t launch_bound32;      /* the same for the FP32 SpMV */
} rafem_mesh_stats;

/* Build a mesh on the current device.
 *   xyz_h      [n_nodes * 3] host, node coordinates (x, y, z) in metres
 *   conn_h     [n_elems * npe] host; hex local order (0,0,0),(1,0,0),(1,1,0),(0,1,0),
 *              (0,0,1),(1,0,1),(1,1,1),(0,1,1) of the reference cube; tets positively oriented
 *   dir_ids_h  [n_dir] host, Dirichlet node ids, strictly increasing; n_dir may be 0
 *   out        receives the handle
 * Every element must have positive Jacobian determinant at its quadrature points
 * (E_MESH otherwise).  Allocates all device memory the other calls use. */
rafem_status rafem_mesh_create(int64_t n_nodes, int64_t n_elems, int32_t npe,
                               const double* xyz_h, const int32_t* conn_h,
                               const int32_t* dir_ids_h, int64_t n_dir, rafem_mesh* out);

/* A batch of independent problems (the ensemble workload: many tissue-parameter samples
 * on meshes of different sizes) as one handle.  Sample q's arrays are as for
 * rafem_mesh_create; the handle holds their disjoint union: sample q's nodes occupy
 * [node_off[q], node_off[q] + n_nodes[q]) of every node vector, followed by padding nodes
 * up to node_off[q+1] (a multiple of 1024, so no GPU workgroup spans two samples); its
 * elements occupy [elem_off[q], elem_off[q+1]) of every element vector; its Dirichlet
 * values occupy [dir_off[q], dir_off[q] + n_dir[q]) of dir_V / dir_T, followed by the
 * values of its padding nodes (isolated Dirichlet nodes; any value, e.g. 0).  Every
 * solve of rafem_step / rafem_step_vjp on a batch handle runs all samples together with
 * per-sample scalars and convergence (each sample's iterates are those of its own solve)
 * and its iteration chunks are replayed as HIP graphs.  Query the layout with
 * rafem_mesh_sample_layout and per-sample results with rafem_sample_info. */
rafem_status rafem_mesh_create_batch(int32_t n_samples, const int64_t* n_nodes,
                                     const int64_t* n_elems, int32_t npe,
                                     const double* const* xyz_h, const int32_t* const* conn_h,
                                     const int32_t* const* dir_ids_h, const int64_t* n_dir,
                                     rafem_mesh* out);

/* node_off, elem_off, dir_off: [n_samples + 1] host outputs (any may be NULL).  A mesh made
 * by rafem_mesh_create is one sample: {0, n_nodes}, {0, n_elems}, {0, n_dir}. */
rafem_status rafem_mesh_sample_layout(rafem_mesh mesh, int64_t* node_off, int64_t* elem_off,
                                      int64_t* dir_off);

/* Use (nonzero) or not HIP graphs for the PCG iteration chunks of this mesh's steps.  On by
 * default for batch handles, and for rafem_step's solves on single meshes of at most 262,144
 * nodes, whose iterations are launch-bound (a call here replaces that rule).  Graphs are not
 * used while SpMV profiling is enabled; they never change a result. */
rafem_status rafem_mesh_set_graphs(rafem_mesh mesh, int32_t enable);

/* Device-driven solves (on by default for batch handles, off for single meshes): each of
 * rafem_step's two solves is enqueued at once -- the PCG iterations and, in mixed
 * precision, every refinement with its inner solve -- each (inner) solve with an iteration
 * budget of ceil(budget_scale x the larger of its counts in the last two solves of its
 * kind) + 3 (kernels past convergence exit at once), and in mixed precision the residual
 * check of one refinement more than the last solve needed.  The solver states are logged on
 * the device after every (inner) solve, and one poll at the end of the solve reads them: it
 * is accepted if it did exactly what the host-driven solve does (every inner solve finished
 * within its budget, every sample converged, no refinement stagnated); otherwise its
 * starting point is restored and it runs host-driven.  Either way the results are bit for
 * bit the host-driven solve's; an accepted solve synchronises with the host once (two per
 * coupled step) instead of at every poll.  Solves without counts from the last two solves of
 * the same kind and precision started the same way (the same predictor order: at the start
 * of a trajectory the order, and with it the counts, still change), and solves while SpMV
 * profiling or region timing is on, run host-driven; so do rafem_step_pc, rafem_step_mono
 * and rafem_step_vjp.
 *   enable        nonzero: on (allocates the solver logs and a copy of one node vector on
 *                 first use)
 *   budget_scale  0 for the default 1.05, else (0, 16] */
rafem_status rafem_mesh_set_device_driven(rafem_mesh mesh, int32_t enable, double budget_scale);

/* Free a mesh and its device memory (synchronises the device first).  NULL is a no-op. */
rafem_status rafem_mesh_destroy(rafem_mesh mesh);

rafem_status rafem_mesh_get_stats(rafem_mesh mesh, rafem_mesh_stats* out);

/* ---------------------------------------------------------------------------
 * Assembly (Sec. III-A: element equations gathered into the global CSR matrix).
 * ------------------------------------------------------------------------- */

/* A = sum_e (mass_coef[e] M_e + stiff_coef[e] K_e) on the mesh's CSR structure,
 * with consistent mass M_e and stiffness K_e of the element (hex: 2x2x2 Gauss;
 * tet: exact), assembled element-parallel colour by colour (no atomics).
 * If dir_vals_d is given, Dirichlet conditions on the mesh's Dirichlet nodes are
 * applied by symmetric lifting that keeps the structure: rhs_lift[f] =
 * -sum_{d in D} A_fd g_d on free rows, rhs_lift[d] = g_d on Dirichlet rows; then
 * rows and columns of D are zeroed (entries stay stored) and A_dd = 1.
 * The right-hand side of the lifted system is b_phys (zero on D) + rhs_lift.
 *   mass_coef_d   [n_elems] device, or NULL for zero
 *   stiff_coef_d  [n_elems] device, or NULL for zero
 *   dir_vals_d    [n_dir] device, values on the Dirichlet nodes in dir_ids order, or NULL
 *                 for no lifting
 *   row_ptr_d     [n_nodes + 1] device output of the structure, or NULL
 *   col_idx_d     [nnz] device output of the structure, or NULL
 *   vals_d        [nnz] device output, FP64 values (required)
 *   vals32_d      [nnz] device output, FP32 copy of the values, or NULL
 *   rhs_lift_d    [n_nodes] device output, or NULL (required if dir_vals_d is given) */
rafem_status rafem_assemble_csr(rafem_mesh mesh, const double* mass_coef_d,
                                const double* stiff_coef_d, const double* dir_vals_d,
                                int32_t* row_ptr_d, int32_t* col_idx_d, double* vals_d,
                                float* vals32_d, double* rhs_lift_d, void* stream);

/* ---------------------------------------------------------------------------
 * Solve (Sec. II-B: CG for SPD systems, with a preconditioner).
 * ------------------------------------------------------------------------- */
#define RAFEM_FP64   0  /* FP64 Jacobi-PCG */
#define RAFEM_MIXED  1  /* FP32-value / FP32-vector inner PCG inside FP64 iterative refinement */

typedef struct {
    double  tol;         /* stop when ||b - A x||_2 <= tol ||b||_2 (recursive residual in FP64 PCG,
                            FP64 true residual of the refinement in MIXED) */
    int32_t maxit;       /* limit on (inner) PCG iterations per solve; <= 0 means 20000 */
    int32_t precision;   /* RAFEM_FP64 or RAFEM_MIXED */
    double  inner_tol;   /* MIXED: relative tolerance of each inner solve (0 means 3e-5); an
                            inner solve stops earlier when a tenth of the reduction the FP64
                            tolerance still needs is reached (the last refinement) */
    int32_t max_outer;   /* MIXED: refinement limit (<= 0 means 30) */
    int32_t poll_every;  /* iterations enqueued between host polls (<= 0 means adaptive) */
    int32_t restart_inner; /* MIXED: 0 (default): after each refinement the inner FP32
                            recurrence goes on from the new FP64 residual with its search
                            direction kept (a reliable update); 1: every refinement starts a
                            new inner Krylov space (plain iterative refinement) */
    int32_t pad;
} rafem_solve_opts;

typedef struct {
    int32_t status;      /* RAFEM_OK, RAFEM_E_NOCONV or RAFEM_E_BREAKDOWN */
    int32_t iters;       /* PCG iterations (FP64) or total inner iterations (MIXED) */
    int32_t outer;       /* refinement steps (MIXED), 0 for FP64 */
    int32_t launched;    /* iterations enqueued, including ones skipped after convergence */
    double  relres;      /* residual norm the stopping test saw, over ||b|| */
    double  relres_true; /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
} rafem_solve_info;

/* Solve A x = b with Jacobi-PCG, x holding the initial guess on entry.
 * A is any square CSR matrix with n_nodes rows, sorted or unsorted columns,
 * a nonzero diagonal and symmetric positive definite values (not checked).
 *   row_ptr_d, col_idx_d, vals_d  CSR of A on the device (int32, int32, FP64)
 *   vals32_d   FP32 copy of vals (required for RAFEM_MIXED, ignored otherwise)
 *   b_d        [n_nodes] right-hand side
 *   x_d        [n_nodes] in: initial guess, out: solution (last iterate on failure)
 *   opts       NULL for defaults (tol 1e-10, FP64)
 *   info       NULL or receives iteration counts and residuals
 * The mesh handle provides the workspaces.  Returns info->status. */
rafem_status rafem_solve(rafem_mesh mesh, const int32_t* row_ptr_d, const int32_t* col_idx_d,
                         const double* vals_d, const float* vals32_d, const double* b_d,
                         double* x_d, const rafem_solve_opts* opts, rafem_solve_info* info,
                         void* stream);

/* The result of rafem_solve_enqueue, written to device memory by its last kernel. */
typedef struct {
    int32_t status;      /* RAFEM_OK; RAFEM_E_NOCONV when the enqueued budget ran out first;
                            RAFEM_E_BREAKDOWN */
    int32_t iters;       /* PCG iterations (FP64) or total inner iterations (MIXED) */
    int32_t outer;       /* refinement steps (MIXED), 0 for FP64 */
    int32_t pad;
    double  relres_true; /* ||b - A x||_2 / ||b||_2 of the returned x, recomputed in FP64 */
} rafem_device_info;

/* rafem_solve with its result kept on the device (Sec. III-A: the solution stays on the
 * device; here the solver's report too): the whole solve is enqueued on `stream` at once
 * and the call returns without synchronising with the host, so that a caller can chain
 * further work, or capture the solve in a graph, and read info_d when it needs it.  With no
 * host poll inside, the budget is fixed beforehand:
 *   FP64:  `iterations` PCG iterations;
 *   MIXED: `refinements` refinement steps, each with an inner solve of at most `iterations`
 *          FP32 iterations, then the residual check of the last one.
 * Iterations and refinements enqueued past convergence exit at their first instruction
 * (each still costs a launch of a few microseconds), so budgets near the expected counts
 * are cheapest.  While the budget suffices the iterates are those of rafem_solve with the
 * same options; a MIXED solve whose refinement stagnates is not handed to FP64 PCG as
 * rafem_solve does, it ends with RAFEM_E_NOCONV.
 *   iterations   [1, 100000]
 *   refinements  MIXED: [1, 14]; ignored for FP64
 *   info_d       device, receives the rafem_device_info (stream-ordered)
 * Other arguments as for rafem_solve.  The first call on a handle allocates the solver-state
 * logs it shares with rafem_mesh_set_device_driven.  Single-mesh handles only (E_ARG on a
 * batch).  Argument errors are returned before anything is enqueued; numerical outcomes
 * only reach info_d. */
rafem_status rafem_solve_enqueue(rafem_mesh mesh, const int32_t* row_ptr_d,
                                 const int32_t* col_idx_d, const double* vals_d,
                                 const float* vals32_d, const double* b_d, double* x_d,
                                 const rafem_solve_opts* opts, int32_t iterations,
                                 int32_t refinements, rafem_device_info* info_d, void* stream);

/* Allocation-free variant of rafem_solve, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): no mesh handle; the solver's
 * workspace (r, p, A p, D^-1, their FP32 twins, partial sums, solver states) lives in one
 * file-scope device array of RAFEM_NOALLOC_SCRATCH_BYTES bytes, which every GPU the library
 * runs on holds from the first such call until the process ends.  The same kernels and
 * launch shapes as rafem_solve on a handle of the same n_rows and nnz, so the iterates are
 * the same.  Calls no hipMalloc / hipFree / pinned-host allocation.  Calls on one device are
 * serialised (each blocks until its solve has finished); the array keeps the last call's
 * contents, and every value a solve reads from it is written by that solve first.
 *   n_rows    rows of A, 1 .. RAFEM_NOALLOC_MAX_ROWS (E_ARG beyond)
 *   nnz       entries of A (row_ptr_d[n_rows]), n_rows .. INT32_MAX
 *   other arguments as rafem_solve (CSR on the device; vals32_d required for RAFEM_MIXED)
 * Returns info->status. */
#define RAFEM_NOALLOC_MAX_ROWS      1048576
#define RAFEM_NOALLOC_SCRATCH_BYTES 63705088
rafem_status rafem_solve_noalloc(int64_t n_rows, int64_t nnz, const int32_t* row_ptr_d,
                                 const int32_t* col_idx_d, const double* vals_d,
                                 const float* vals32_d, const double* b_d, double* x_d,
                                 const rafem_solve_opts* opts, rafem_solve_info* info,
                                 void* stream);

/* Adjoint solve A^T lambda = g for a matrix assembled by rafem_assemble_csr.
 * The lifted matrices are symmetric, so this runs the same PCG on A with the
 * right-hand side g with its Dirichlet rows zeroed (the adjoint of a prescribed
 * value is zero).  Arguments as rafem_solve; g_d [n_nodes] is not modified;
 * lambda_d [n_nodes] holds the initial guess on entry and the solution on exit. */
rafem_status rafem_solve_adjoint(rafem_mesh mesh, const int32_t* row_ptr_d,
                                 const int32_t* col_idx_d, const double* vals_d,
                                 const float* vals32_d, const double* g_d, double* lambda_d,
                                 const rafem_solve_opts* opts, rafem_solve_info* info,
                                 void* stream);

/* y = A x on the device, with the same kernel the FP64 solver uses
 * (the FP32 one when vals_d is NULL and vals32_d, x32_d, y32_d are given).
 * Returns without synchronising.  Mainly for measurement and tests. */
rafem_status rafem_spmv(rafem_mesh mesh, const int32_t* row_ptr_d, const int32_t* col_idx_d,
                        const double* vals_d, const double* x_d, double* y_d,
                        const float* vals32_d, const float* x32_d, float* y32_d, void* stream);

/* The product of a time step's solves, y = A x, run by the very kernels the PCG
 * iterations use on the mesh's own slab layout (Sec. III-A: the solve of the assembled
 * system; Sec. III-B: the structure analysed once per mesh): 64-row slabs with shared
 * column offsets, 16-bit or 32-bit per-row column offsets, the tuned slab shape, launch
 * bound and value loads, and the dot product x.(A x) fused into the product.
 *   matrix     0: the potential matrix, 1: the bioheat matrix, as the last rafem_step (or
 *              rafem_step_pc / rafem_step_vjp) on this handle assembled them, Dirichlet
 *              rows and columns lifted (E_STATE before such a step)
 *   precision  RAFEM_FP64: x_d, y_d are double [n_nodes] and the FP64 values are used;
 *              RAFEM_MIXED: x_d, y_d are float [n_nodes], FP32 values (the inner PCG's kernel)
 *   b_d        NULL, or (FP64 only) double [n_nodes]: then y = b - A x with the kernel of
 *              the refinement residual instead
 *   dots_h     NULL, or host output, blocking: without b, [n_samples] sums x.(A x) of each
 *              sample, from the kernel's per-group partials added in slot order; with b,
 *              [2 n_samples] pairs (||b - A x||^2, ||b||^2) as the solver state holds them
 * Node vectors use the handle's layout (a batch handle: every sample with its padding).
 * Returns without synchronising when dots_h is NULL.  Uses the handle's check-state and
 * partial-sum workspace, so it must not overlap a solve on the same handle. */
rafem_status rafem_spmv_step(rafem_mesh mesh, int32_t matrix, int32_t precision, const void* x_d,
                             void* y_d, const double* b_d, double* dots_h, void* stream);

/* ---------------------------------------------------------------------------
 * Measurement.  While enabled, the SpMV kernel of every PCG iteration that the solves
 * on this mesh enqueue carries a pair of HIP events stamped when the kernel itself
 * starts and ends (at most 2048 per chunk of iterations; the gap before a launch is not
 * counted); after each chunk the durations of the launches that performed an iteration
 * are accumulated, launches skipped after convergence are not.  Iteration chunks are not
 * replayed as graphs meanwhile.  Enabling creates the events, disabling destroys them.
 * ------------------------------------------------------------------------- */
rafem_status rafem_profile_enable(rafem_mesh mesh, int32_t enable);

/* Timing of the PCG SpMV kernel (with its fused p.Ap) on this mesh's potential matrix as
 * the last rafem_step assembled it (E_STATE before any step).  n_copies >= 1 copies of
 * its values (FP64, or FP32 for RAFEM_MIXED) are made and reps launches rotate through
 * them, so that with enough copies no launch finds its values in the 256 MB Infinity
 * Cache; each launch is timed by events stamped at the kernel's own start and end.
 * mean_us receives the mean duration.  Allocates and frees the copies (E_NOMEM if they do
 * not fit) and synchronises; a measurement call, not part of a step. */
rafem_status rafem_spmv_timing(rafem_mesh mesh, int32_t precision, int32_t n_copies,
                               int32_t reps, double* mean_us);

/* Mean duration in microseconds and number of the SpMV launches measured since the
 * last reset, for the FP64 kernel (precision RAFEM_FP64) or the FP32 kernel of the
 * inner iterations (RAFEM_MIXED).  reset != 0 clears the accumulators after reading. */
rafem_status rafem_profile_read(rafem_mesh mesh, int32_t precision, double* mean_us,
                                int64_t* count, int32_t reset);

/* ---------------------------------------------------------------------------
 * Region timing, the breakdown of a time step into the paper's traced regions (Sec. III-C,
 * Fig. 11: assembly, solve, and the copies of the convergence check).  When enabled, each
 * rafem_step, rafem_step_pc and rafem_step_mono call records HIP events on its stream at
 * the boundaries of its regions and, once the step has finished, adds the device time of
 * every interval to its region.  Off by default (the events cost a few microseconds).
 * ------------------------------------------------------------------------- */
typedef struct {
    double  assembly_ms;  /* matrix / Jacobian assembly, lifting, right-hand sides */
    double  solve_ms;     /* linear solves (PCG, mixed refinement, GMRES) with their polls */
    double  check_ms;     /* corrector convergence checks, state copies, predictor */
    int64_t steps;        /* step calls measured */
} rafem_regions;

rafem_status rafem_regions_enable(rafem_mesh mesh, int32_t enable);
/* Accumulated times since the last reset (reset != 0 clears them after reading). */
rafem_status rafem_regions_read(rafem_mesh mesh, rafem_regions* out, int32_t reset);

/* ---------------------------------------------------------------------------
 * One coupled time step (Sec. II-A, Fig. 1: assemble + solve for voltage and heat).
 * ------------------------------------------------------------------------- */
typedef struct {
    double  rho_c;        /* volumetric heat capacity [J/m^3/K] */
    double  dt;           /* time step [s] */
    double  T_a;          /* arterial temperature of the perfusion term [C] */
    double  alpha_sigma;  /* sigma = sigma0 (1 + alpha_sigma (Tbar_e - T_ref)) */
    double  T_ref;
    int32_t coupled;      /* 0: bioheat step only, with zero Joule source and V untouched */
    int32_t reuse_bioheat;/* nonzero: reuse the bioheat matrix assembled by the previous call
                             (k, perfusion, rho_c unchanged); E_STATE if there is none; a
                             matrix built for another dt is rebuilt regardless */
    int32_t extrapolate;  /* rafem_step of a coupled problem only.  1: this call continues the
                             trajectory of the previous rafem_step call on this handle: both
                             solves start from the polynomial extrapolation in time of the
                             states kept from the trajectory's calls (sigma and the right-hand
                             side still use T^n): the Lagrange polynomial through (t_n, T^n),
                             (t_n - h1, T^{n-1}), ..., (t_n - h1 - ... - hq, T^{n-q}) taken at
                             t_n + dt, h_k being the dt of the k-th previous call, q the lesser
                             of extrapolate_order and the number of earlier states kept (up to 4);
                             the same for V.  q = 1 is T^n + (dt/h1)(T^n - T^{n-1}).  2: a new
                             trajectory starts here (solves start from T_d, V_d; the states are
                             kept for the next call).  0: off.  A call with 0, a failed call,
                             rafem_step_pc and rafem_step_mono end the trajectory (the next call
                             with 1 then behaves as 2).  Other values: E_ARG.
                             rafem_step_vjp: 1: this call continues the reverse sweep of the
                             previous rafem_step_vjp call on this handle: its adjoint solves
                             start from that call's mu and nu (the adjoint states of the step
                             after this one); 2: a sweep starts here (solves start from zero;
                             mu and nu are kept for the next call); 0: from zero, nothing kept.
                             The solves run to the same tolerance either way. */
    int32_t extrapolate_order; /* 1 (linear; also 0) .. 4 (quartic); other values: E_ARG */
} rafem_phys;

typedef struct {
    rafem_solve_info V;   /* potential solve (zeroed if not coupled) */
    rafem_solve_info T;   /* bioheat solve */
} rafem_step_info;

/* Advance (T^n, V^n) to (T^{n+1}, V^{n+1}):
 *   sigma_e = sigma0_e (1 + alpha (mean of T^n over the element - T_ref));
 *   [sum_e sigma_e K_e] V = 0 with V = dir_V on D                      (potential);
 *   F_i = sum_e int N_i sigma_e grad V . grad V                         (Joule source);
 *   [sum_e (rho_c/dt + perf_e) M_e + k_e K_e] T^{n+1}
 *        = (rho_c/dt) M T^n + T_a sum_e perf_e M_e 1 + F,  T = dir_T on D  (bioheat).
 *   k_e_d, perf_e_d, sigma0_e_d  [n_elems] device
 *   dir_V_d, dir_T_d             [n_dir] device, values on D in dir_ids order
 *   T_d  [n_nodes] in: T^n, out: T^{n+1}
 *   V_d  [n_nodes] in: initial guess (previous potential), out: V^{n+1}
 *   opts applies to both solves (NULL: tol 1e-12, FP64). */
rafem_status rafem_step(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                        const double* perf_e_d, const double* sigma0_e_d,
                        const double* dir_V_d, const double* dir_T_d, double* T_d, double* V_d,
                        const rafem_solve_opts* opts, rafem_step_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Predictor-corrector step (the application's main loop, Sec. II-A and Fig. 1: each
 * time step extrapolates the solution, then repeats the corrector -- element equations
 * with updated values, assembly, solve -- until a convergence threshold is met; a step
 * whose corrector has not converged after the allowed iterations is not accepted and is
 * retried with half the step, Sec. IV).
 * ------------------------------------------------------------------------- */

typedef struct {
    double  tol;         /* corrector threshold on ||T^{k+1} - T^k||_2 / ||T^{k+1}||_2 (<= 0: 1e-10) */
    int32_t max_iters;   /* corrector iterations before the step is rejected (<= 0: 50) */
} rafem_corrector_opts;

typedef struct {
    int32_t accepted;     /* 1: T and V advanced to t + dt; 0: left at t (rejected or failed) */
    int32_t iters;        /* corrector iterations performed */
    double  change;       /* last relative change of T */
    int32_t solver_iters; /* PCG iterations (inner iterations if MIXED) of all solves */
    int32_t status;       /* RAFEM_OK unless a solve failed */
} rafem_corrector_info;

/* One predictor-corrector step of size phys->dt on a single mesh.
 *   predictor  T* = T^n + (dt / dt_prev)(T^n - T^{n-1}), or T^n when T_prev_d is NULL;
 *   corrector  k = 1, 2, ...: sigma from T^{n+1,k} (T^{n+1,0} = T*), potential solve (V
 *              warm-started from its last value), Joule load, bioheat solve with T^n on the
 *              right-hand side giving T^{n+1,k+1}; stop when the relative change of T is
 *              <= copts->tol (accepted) or after copts->max_iters iterations (rejected).
 * The first corrector iterate from T* = T^n is exactly rafem_step.  The bioheat matrix is
 * reassembled when dt differs from the one it was built for (or reuse_bioheat is 0).
 *   T_prev_d [n_nodes] device or NULL; dt_prev its step (> 0 when T_prev_d is given)
 *   T_d, V_d [n_nodes] device, in: T^n, V^n; out: T^{n+1}, V^{n+1} if accepted, unchanged
 *            otherwise
 * Returns RAFEM_OK for accepted and rejected steps alike (see info->accepted), a solve's
 * status if one failed (T_d, V_d then restored).  E_ARG on a batch handle. */
rafem_status rafem_step_pc(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                           const double* perf_e_d, const double* sigma0_e_d,
                           const double* dir_V_d, const double* dir_T_d, const double* T_prev_d,
                           double dt_prev, double* T_d, double* V_d, const rafem_solve_opts* opts,
                           const rafem_corrector_opts* copts, rafem_corrector_info* info,
                           void* stream);

/* ---------------------------------------------------------------------------
 * Monolithic corrector.  The paper's corrector assembles the element equations, with the
 * latest values, into one global matrix with two unknowns per node (temperature and
 * potential; matrix order = 2 x nodes, Table II) that is sparse and structurally
 * symmetric, and solves it with restarted GMRES(m) (Sec. II-A, Sec. II-B, Sec. III-B,
 * Fig. 3).  Here that matrix is the Jacobian J of the implicit coupled step
 *   R_T = sum_e [(rho_c/dt + perf_e) M_e + k_e K_e] T_e - M_e ((rho_c/dt) T^n_e + perf_e T_a)
 *         - f_e(sigma_e(T), V_e),
 *   R_V = sum_e sigma_e(T) K_e V_e,   sigma_e(T) = sigma0_e (1 + alpha (mean_e T - T_ref)),
 * at the free nodes (f_e: Joule loads int N sigma grad V . grad V), 0 at Dirichlet nodes;
 * its element blocks (c_e = sigma0_e alpha / npe, q_e = f_e at sigma = 1, 1 = all ones):
 *   dR_T/dT = (rho_c/dt + perf_e) M_e + k_e K_e - c_e q_e 1^T,   dR_T/dV = -df_e/dV_e,
 *   dR_V/dT = c_e (K_e V_e) 1^T,                                dR_V/dV = sigma_e K_e,
 * Dirichlet rows and columns replaced by the identity's.  Unknown 2i is T_i, 2i+1 is V_i.
 * One corrector iteration is one Newton step J delta = -R; its root is the fixed point of
 * the staggered corrector of rafem_step_pc.  All three calls below need a single-mesh
 * handle (E_ARG on a batch) and phys->coupled != 0.
 * ------------------------------------------------------------------------- */

#define RAFEM_GMRES_MAX_M 200

typedef struct {
    int32_t m;           /* Krylov vectors per restart cycle, 1..RAFEM_GMRES_MAX_M (<= 0: 30) */
    int32_t max_iters;   /* Arnoldi steps over all cycles (<= 0: 20000) */
    double  tol;         /* stop when ||b - J x||_2 <= tol ||b||_2 (<= 0: 1e-10) */
    int32_t precision;   /* RAFEM_FP64, or RAFEM_MIXED: the Arnoldi process on FP32 copies of
                            J, the basis and the block inverses (FP64 sums), while every
                            restart forms the true residual b - J x and the update in FP64 */
    int32_t pad;
} rafem_gmres_opts;

typedef struct {
    int32_t status;      /* RAFEM_OK, E_NOCONV (max_iters reached), E_BREAKDOWN (non-finite
                            value or singular Hessenberg) */
    int32_t iters;       /* Arnoldi steps over all cycles */
    int32_t cycles;      /* restart cycles */
    int32_t pad;
    double  relres;      /* last Givens-rotated residual estimate / ||b|| */
    double  relres_true; /* ||b - J x|| / ||b|| at the last restart (the exit) */
} rafem_gmres_info;

/* The Jacobian and residual at the state (T, V), for inspection and tests.
 *   T_n_d, T_d, V_d  [n_nodes] device: T^n, and the iterate (T, V), which must carry the
 *                    Dirichlet values
 *   planes_d  [4 nnz] device out: TT, TV, VT, VV values, each plane in the CSR order of
 *             rafem_csr_structure (zero-filled first)
 *   R_d       [2 n_nodes] device out: R interleaved (R[2i] = R_T,i, R[2i+1] = R_V,i)
 * Allocates nothing beyond the handle's step buffers. */
rafem_status rafem_mono_jacobian(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                                 const double* perf_e_d, const double* sigma0_e_d,
                                 const double* T_n_d, const double* T_d, const double* V_d,
                                 double* planes_d, double* R_d, void* stream);

/* Assemble J and R at (T, V) as above and solve J delta = -R from delta = 0 by restarted
 * GMRES(opts->m) with right preconditioning by the inverses of J's 2x2 diagonal node
 * blocks (classical Gram-Schmidt applied twice, Givens rotations; a cycle stops when the
 * rotated residual meets opts->tol, a restart recomputes the true residual).
 *   delta_d  [2 n_nodes] device out: the update, interleaved like R
 *   hist_d   [hist_len] device out or NULL: the rotated residual estimate / ||R|| after
 *            every Arnoldi step (the first hist_len steps)
 * Returns info->status.  The first call allocates the handle's monolithic workspace:
 * 32 B per matrix slot plus (m + 5) vectors of 16 B per node. */
rafem_status rafem_mono_solve(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                              const double* perf_e_d, const double* sigma0_e_d,
                              const double* T_n_d, const double* T_d, const double* V_d,
                              const rafem_gmres_opts* opts, double* delta_d, double* hist_d,
                              int32_t hist_len, rafem_gmres_info* info, void* stream);

typedef struct {
    int32_t accepted;     /* 1: T and V advanced to t + dt; 0: left at t (rejected or failed) */
    int32_t iters;        /* Newton (corrector) iterations performed */
    double  change;       /* last ||delta_T|| / ||T|| */
    int32_t gmres_iters;  /* Arnoldi steps of all linear solves */
    int32_t gmres_cycles; /* restart cycles of all linear solves */
    int32_t status;       /* RAFEM_OK unless a linear solve failed */
    int32_t pad;
    double  relres_true_max; /* largest exit residual of the linear solves */
} rafem_mono_info;

/* One predictor-corrector step of size phys->dt with the monolithic corrector: the
 * predictor of rafem_step_pc gives T*, the iterate starts at (T*, V^n) with the Dirichlet
 * values imposed, and Newton steps (each solved as in rafem_mono_solve) run until
 * ||delta_T|| <= copts->tol ||T|| (accepted) or copts->max_iters steps (rejected).
 *   T_prev_d, dt_prev, T_d, V_d, copts: as for rafem_step_pc
 * Returns RAFEM_OK for accepted and rejected steps alike, a solve's status if one failed
 * (T_d, V_d then restored). */
rafem_status rafem_step_mono(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                             const double* perf_e_d, const double* sigma0_e_d,
                             const double* dir_V_d, const double* dir_T_d,
                             const double* T_prev_d, double dt_prev, double* T_d, double* V_d,
                             const rafem_gmres_opts* opts, const rafem_corrector_opts* copts,
                             rafem_mono_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Reverse mode: gradients of a loss on the final temperature with respect to the
 * per-element conductivity k_e and perfusion w_e, by the discrete adjoint of the
 * steps above run backwards in time (the time loop of Sec. II-A, reversed).
 * ------------------------------------------------------------------------- */

/* Reverse of one rafem_step.  Given the adjoint load lambda on T^n (dL/dT^n), computes
 *   A_T mu = lambda (Dirichlet rows zeroed), K_sigma(T^{n-1}) nu = (dF/dV)^T mu,
 *   grad_k[e] += -mu_e^T K_e T^n_e,  grad_perf[e] += -mu_e^T M_e (T^n_e - T_a),
 * and overwrites lambda with the adjoint load on T^{n-1}:
 *   (rho_c/dt) M mu + sum_e (mu_e^T J_e(V^n) - nu_e^T K_e V^n_e) sigma0_e alpha / npe
 * on the nodes of e (J_e = Joule load at unit conductivity).  Both matrices are
 * symmetric, so the adjoint solves are PCG solves on the same matrices.
 *   T_prev_d, V_d, T_d  [n_nodes] device: T^{n-1}, V^n, T^n of the forward step
 *   lambda_d            [n_nodes] device, in: dL/dT^n; out: dL/dT^{n-1}
 *   grad_k_d, grad_perf_d [n_elems] device, accumulated (+=)
 *   other arguments as rafem_step; phys->reuse_bioheat as there; info->T describes the
 *   mu solve and info->V the nu solve (zero when not coupled). */
rafem_status rafem_step_vjp(rafem_mesh mesh, const rafem_phys* phys, const double* k_e_d,
                            const double* perf_e_d, const double* sigma0_e_d,
                            const double* dir_V_d, const double* dir_T_d, const double* T_prev_d,
                            const double* V_d, const double* T_d, double* lambda_d,
                            double* grad_k_d, double* grad_perf_d, const rafem_solve_opts* opts,
                            rafem_step_info* info, void* stream);

/* Lesion-temperature loss L = scale * sum_k (T[ids[k]] - target[k])^2 and its gradient
 * grad = dL/dT (2 scale (T - target) on ids, 0 elsewhere), deterministically summed.
 *   ids_d [n_loss] device node ids (distinct), target_d [n_loss] device
 *   T_d [n_nodes] device; loss_d [1] device output; grad_d [n_nodes] device output or NULL */
rafem_status rafem_lesion_loss(rafem_mesh mesh, int64_t n_loss, const int32_t* ids_d,
                               const double* target_d, const double* T_d, double scale,
                               double* loss_d, double* grad_d, void* stream);

/* Per-sample solve information of the last rafem_step on this mesh (sample in
 * [0, n_samples)); for a single mesh, sample 0 repeats the step's own info.  For a
 * mixed-precision solve, iters counts that sample's FP32 inner iterations (plus FP64
 * iterations if it fell back) and outer its refinements (negative: the refinement
 * stagnated and FP64 PCG finished the sample). */
rafem_status rafem_sample_info(rafem_mesh mesh, int32_t sample, rafem_step_info* out);

#ifdef __cplusplus
}
#endif

#endif /* RAFEM_H */
