// Jacobi-PCG kernels for gfx950 (CDNA4, wave64), for one system or a batch of
// independent systems solved together.
//
// A batch is the union of S systems with disjoint rows: sample s owns rows
// [row_off[s], row_off[s+1]), and every interior offset is a multiple of kRowAlign, so
// no workgroup of any kernel spans two samples.  Each sample has its own solver state
// (scalars, tolerance, iteration count, done flag); kernels look up the sample of their
// first row, skip work once that sample is done, and reduce dot products per sample.
//
// Reductions are deterministic and need no atomics or fences: every block stores its
// partial sums in a fixed slot, and the consumer (every block of the next kernel, or a
// one-block-per-sample finalize kernel) adds the slots of its sample in index order
// after the kernel boundary, so all consumers of a sample hold bit-identical scalars.
// The iteration index lives in device memory (`itb` plus the iteration's offset j in
// its chunk, advanced by k_advance after a chunk), so a chunk of iterations can be
// captured once in a graph and replayed.  Scalars carried between iterations are kept
// in slots chosen by the iteration's parity, so no kernel reads a slot it writes.
//
// The SpMV kernels stream the matrix in one of two layouts:
//   * CSR, LANES consecutive lanes per row (general matrices handed over the ABI);
//   * SELL with 64-row slabs, one row per lane (the step path): entry j of a slab's 64
//     rows is one contiguous wavefront load.  Most slabs of the grid meshes share one
//     column-offset list for all their rows (read through the scalar cache; the x reads
//     of an entry are then 64 consecutive words); the others keep per-lane column
//     offsets, as int16 distances to the row when they fit.
// Workgroups walk contiguous row ranges, remapped so each XCD (own L2) takes one
// contiguous share of the rows.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "fem_device.hpp"
#include "internal.hpp"

namespace rafem {
namespace {

using namespace dev;

// Sample owning `row` (largest s with row_off[s] <= row): one load from the table of the
// sample of every kRowAlign-row block (sample boundaries are multiples of kRowAlign), or a
// binary search over row_off when there is no table.
__device__ __forceinline__ int sample_of(const Samples& B, int row) {
    if (B.S == 1) return 0;
    if (B.tab) return B.tab[row / kRowAlign];
    int lo = 0, hi = B.S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.row_off[mid] <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Partial slots [b0, b1) that a producer with `rpb` rows per block wrote for sample s.
__device__ __forceinline__ void sample_blocks(const Samples& B, int s, int rpb, int& b0,
                                              int& b1) {
    b0 = B.row_off[s] / rpb;
    b1 = (B.row_off[s + 1] + rpb - 1) / rpb;
}

// Fixed-order totals of partial slots [b0, b1) of K arrays; returned to every thread.
// Thread t adds slots b0 + t + WG u in increasing u (the order depends only on the offset
// from b0, so a sample sums alike in any batch), then the block adds the threads.  The
// slots come from the previous kernel (other XCDs' L2s): kRangeUnroll of them are loaded
// at once so their latencies overlap.
constexpr int kRangeUnroll = 8;

// The first batch of a thread's slots, loaded ahead (range_prefetch) so that the vector
// kernels can issue these loads together with their vector loads and before they read the
// solver state; range_totals then adds it and any further batches.
template <int K>
struct RangeBatch {
    double v[K][kRangeUnroll];
};

template <int K>
__device__ __forceinline__ void range_prefetch(const double* __restrict__ partials, int nb,
                                               int b0, int b1, RangeBatch<K>& first) {
    const int base = b0 + (int)threadIdx.x;
#pragma unroll
    for (int u = 0; u < kRangeUnroll; ++u) {
        const int i = base + u * WG;
#pragma unroll
        for (int k = 0; k < K; ++k) first.v[k][u] = i < b1 ? partials[k * nb + i] : 0.0;
    }
}

template <int K>
__device__ __forceinline__ void range_totals(const double* __restrict__ partials, int nb, int b0,
                                             int b1, double (&tot)[K],
                                             const RangeBatch<K>* first = nullptr) {
    __shared__ double bcast[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = 0.0;
    for (int base = b0 + (int)threadIdx.x; base < b1; base += kRangeUnroll * WG) {
        RangeBatch<K> b;
        if (first && base == b0 + (int)threadIdx.x)
            b = *first;
        else
            range_prefetch<K>(partials, nb, base - (int)threadIdx.x, b1, b);
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int u = 0; u < kRangeUnroll; ++u) tot[k] += b.v[k][u];
        }
    }
    block_sum<K>(tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) bcast[k] = tot[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = bcast[k];
}

// ---------------------------------------------------------------------------
// Solver state
// ---------------------------------------------------------------------------
__global__ void k_state_init(PcgState* st, int S, double tol, int maxit, int* itb) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0 && itb) *itb = 0;
    if (s >= S) return;
    PcgState& t = st[s];
    t.rzs[0] = t.rzs[1] = t.pq = t.beta = t.rr = t.bb = 0.0;
    t.tol = tol;
    t.tol2 = 0.0;
    t.scale = 1.0;
    t.scale_prev = 1.0;
    t.rr_first = 0.0;
    t.iters = 0;
    t.maxit = maxit;
    t.done = 0;
    t.status = RAFEM_E_NOCONV;
    t.bad_diag = 0;
}

__global__ void k_advance(int* itb, int k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *itb += k;
}

// dinv = 1 / diag(A) (also as FP32), CSR, one system.  A missing or non-positive
// diagonal marks the state.
__global__ __launch_bounds__(WG) void k_diag_inv(const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const double* __restrict__ v, int n,
                                                 double* __restrict__ dinv,
                                                 float* __restrict__ dinv32, PcgState* st) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d += v[k];
    const double inv = (d > 0.0 && finite(d)) ? 1.0 / d : 0.0;
    if (!(d > 0.0) || !finite(d)) st->bad_diag = 1;
    dinv[i] = inv;
    if (dinv32) dinv32[i] = (float)inv;
}

// ---------------------------------------------------------------------------
// Row kernels
// ---------------------------------------------------------------------------
// [row-kernels-begin] (the text up to the matching end marker is what the recorded byte
// counters of these kernels refer to)
enum RowMode : int {
    ROW_PLAIN = 0,  // y = A x
    ROW_DOT = 1,    // y = A x, partials of x.y (PCG step; skipped once the sample is done)
    ROW_START = 2,  // r = b - A x; y = p = D^-1 r, partials of r.p, r.r, b.b (PCG start)
    ROW_RESID = 3,  // y = b - A x, partials of y.y, b.b (refinement / true residual)
};

template <typename T>
struct RowArgs {
    const int* __restrict__ rp;       // CSR
    const int* __restrict__ ci;
    const int* __restrict__ sptr;     // SELL
    const int* __restrict__ scol;
    const int16_t* __restrict__ sdel;
    const int* __restrict__ sofs;     // shared-offset slabs
    const int* __restrict__ soff;
    const T* __restrict__ val;
    const T* __restrict__ x;
    T* __restrict__ y;
    const double* __restrict__ b;
    const double* __restrict__ dinv;
    double* __restrict__ pout;
    double* partials;
    PcgState* st;
    Samples smp;
    int n;
    int nslabs;
    int rows_per_block;   // CSR: rows per workgroup
    int slabs_per_block;  // SELL: slabs per workgroup
    int outer_mode;
    int resident;         // SELL, streaming kernels: slabs starting below this value slot
                          // read their values with ordinary loads, the others stream them
};

// Per-row epilogue of every row mode; acc receives this lane's dot-product terms.
template <typename T, int MODE>
__device__ __forceinline__ void row_epilogue(const RowArgs<T>& a, int r, T sum, double (&acc)[3]) {
    if constexpr (MODE == ROW_PLAIN) {
        a.y[r] = sum;
    } else if constexpr (MODE == ROW_DOT) {
        a.y[r] = sum;
        acc[0] += (double)a.x[r] * (double)sum;
    } else {
        const double bi = a.b[r];
        const double ri = bi - (double)sum;
        acc[1] += ri * ri;
        acc[2] += bi * bi;
        if constexpr (MODE == ROW_START) {
            // the PCG keeps z = D^-1 r (r itself is formed where a dot product needs it)
            const double zi = a.dinv[r] * ri;
            a.y[r] = (T)zi;
            a.pout[r] = zi;
            acc[0] += ri * zi;
        } else {
            a.y[r] = (T)ri;
        }
    }
}

template <typename T, int MODE>
__device__ __forceinline__ bool skip_sample(const RowArgs<T>& a, int row0) {
    if constexpr (MODE == ROW_DOT) return a.st[sample_of(a.smp, row0)].done != 0;
    if constexpr (MODE == ROW_RESID) return a.outer_mode && a.st[sample_of(a.smp, row0)].done;
    return false;
}

template <int MODE>
__device__ __forceinline__ void row_partials(double (&acc)[3], double* partials, int blk, int nb) {
    if constexpr (MODE == ROW_DOT) {
        double v[1] = {acc[0]};
        store_partials<1>(v, partials, blk, nb);
    } else if constexpr (MODE != ROW_PLAIN) {
        store_partials<3>(acc, partials, blk, nb);
    }
}

template <typename T, int LANES, int MODE>
__global__ __launch_bounds__(WG) void k_csr(RowArgs<T> a) {
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int row0 = blk * a.rows_per_block;
    if (skip_sample<T, MODE>(a, row0)) return;
    const int row1 = min(row0 + a.rows_per_block, a.n);
    const int g = threadIdx.x / LANES, sub = threadIdx.x % LANES;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int r = row0 + g; r < row1; r += WG / LANES) {
        const int s = a.rp[r], e = a.rp[r + 1];
        T sum = T(0);
#pragma unroll 4
        for (int k = s + sub; k < e; k += LANES) sum += a.val[k] * a.x[a.ci[k]];
#pragma unroll
        for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, LANES);
        if (sub == 0) row_epilogue<T, MODE>(a, r, sum, acc);
    }
    row_partials<MODE>(acc, a.partials, blk, nb);
}

constexpr int kSellUnroll = 9;


// Sum over the entries of one row in entry order.  COL is int (absolute columns, xr = x)
// or int16_t (offsets to the row, xr = x + row).
// Entries go in batches of kSellUnroll whose loads are all issued before their x reads; a
// last, shorter batch is masked (its missing entries add nothing), so a row of any width
// keeps a whole batch of loads in flight (the 15-entry rows of the tet meshes: 9 + 6).
// COL is int (absolute columns, xr = x) or int16_t (offsets to the row, xr = x + row).
// A matrix value; NT: a nontemporal load (the values stream through the caches once, which
// pays when the matrix does not fit the Infinity Cache and costs when it does).
template <typename T, bool NT>
__device__ __forceinline__ T load_value(const T* __restrict__ p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T, typename COL, bool MASKED, bool NT>
__device__ __forceinline__ void sell_batch(const COL* __restrict__ cp, const T* __restrict__ vp,
                                           const T* __restrict__ xr, int j, int width, T& sum) {
    int c[kSellUnroll];
    T v[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u) {
        const bool in = !MASKED || j + u < width;
        c[u] = in ? (int)cp[(j + u) * WAVE] : 0;
        v[u] = in ? load_value<T, NT>(vp + (j + u) * WAVE) : T(0);
    }
    T g[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u) g[u] = (!MASKED || j + u < width) ? xr[c[u]] : T(0);
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u)
        if (!MASKED || j + u < width) sum += v[u] * g[u];
}

template <typename T, typename COL, bool NT>
__device__ __forceinline__ T sell_row(const COL* __restrict__ cp, const T* __restrict__ vp,
                                      const T* __restrict__ xr, int width) {
    T sum = T(0);
    int j = 0;
    for (; j + kSellUnroll <= width; j += kSellUnroll)
        sell_batch<T, COL, false, NT>(cp, vp, xr, j, width, sum);
    if (j < width) sell_batch<T, COL, true, NT>(cp, vp, xr, j, width, sum);
    return sum;
}

// The same sum for a shared-offset slab: entry j of every row has column row + off[j],
// off being one list for the whole wavefront (read through the scalar cache), so the x
// reads of one entry are 64 consecutive words.  Same order of operations as sell_row; the
// entries that are not in the matrix hold 0 and add exactly nothing.
template <typename T, bool MASKED, bool NT>
__device__ __forceinline__ void shared_batch(const int* __restrict__ off, const T* __restrict__ vp,
                                             const T* __restrict__ xr, int j, int width, T& sum) {
    int c[kSellUnroll];
    T v[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u) {
        const bool in = !MASKED || j + u < width;
        c[u] = in ? off[j + u] : 0;
        v[u] = in ? load_value<T, NT>(vp + (j + u) * WAVE) : T(0);
    }
    T g[kSellUnroll];
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u) g[u] = (!MASKED || j + u < width) ? xr[c[u]] : T(0);
#pragma unroll
    for (int u = 0; u < kSellUnroll; ++u)
        if (!MASKED || j + u < width) sum += v[u] * g[u];
}

template <typename T, bool NT>
__device__ __forceinline__ T sell_row_shared(const int* __restrict__ off, const T* __restrict__ vp,
                                             const T* __restrict__ xr, int width) {
    T sum = T(0);
    int j = 0;
    for (; j + kSellUnroll <= width; j += kSellUnroll)
        shared_batch<T, false, NT>(off, vp, xr, j, width, sum);
    if (j < width) shared_batch<T, true, NT>(off, vp, xr, j, width, sum);
    return sum;
}

// Partial sums of the SELL kernels cover fixed groups of kSlabGroup slabs, whatever the
// workgroup shape, and are formed in a fixed order (per slab: wavefront butterfly; within
// a group: wavefront w adds its slabs w, w + 4 in that order; then the four wavefronts in
// order).  So the tuned shape (1 or 2 groups per workgroup) never changes a result.
constexpr int kSlabGroup = 2 * NWAVES;
constexpr int kMaxGroups = 2;

template <int K>
__device__ __forceinline__ void store_group_partials(double (&v)[kMaxGroups][K], int ngroups,
                                                     double* partials, int g0, int nb) {
    __shared__ double lds[kMaxGroups][K][NWAVES];
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    for (int g = 0; g < ngroups; ++g) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double t = wave_sum(v[g][k]);
            if (lane == 0) lds[g][k][w] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int g = 0; g < ngroups; ++g) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double t = 0.0;
                for (int j = 0; j < NWAVES; ++j) t += lds[g][k][j];
                partials[k * nb + g0 + g] = t;
            }
        }
    }
}

// One row of a slab, by the slab's column kind.
template <typename T, int COLS, bool NT>
__device__ __forceinline__ T slab_row(const RowArgs<T>& a, int so, int base, int lane, int r,
                                      int width) {
    if (so >= 0)
        return sell_row_shared<T, NT>(a.soff + so, a.val + base + lane, a.x + r, width);
    if (COLS == 1 || (COLS == 2 && so == -1))
        return sell_row<T, int16_t, NT>(a.sdel + base + lane, a.val + base + lane,
                                        a.x + min(r, a.n - 1), width);
    return sell_row<T, int, NT>(a.scol + base + lane, a.val + base + lane, a.x, width);
}

// Column kinds of the slabs without a shared offset list: COLS 0: 32-bit columns, 1: 16-bit
// offsets to the row, 2: either, per slab (sofs -1 / -2).  Separate instantiations keep the
// common layouts' kernels free of the third path (its registers lowered their occupancy).
template <typename T, int MODE, int COLS, bool NT>
__device__ __forceinline__ void sell_rows(const RowArgs<T>& a) {
    const int nblk = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nblk);
    const int s0 = blk * a.slabs_per_block;
    const int lane = threadIdx.x % WAVE;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);  // wave-uniform
    // the wavefront's first slab pointers are read together with the sample state, so
    // the two latencies overlap (sptr has nslabs + 1 entries)
    const int sl0 = min(s0 + w, a.nslabs - 1);
    const int base0 = a.sptr[sl0], end0 = a.sptr[sl0 + 1], so0 = a.sofs[sl0];
    if (skip_sample<T, MODE>(a, s0 * WAVE)) return;
    const int s1 = min(s0 + a.slabs_per_block, a.nslabs);
    double acc[kMaxGroups][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int i = 0; s0 + w + NWAVES * i < s1; ++i) {
        const int sl = s0 + w + NWAVES * i;
        const int base = i == 0 ? base0 : a.sptr[sl];
        const int width = ((i == 0 ? end0 : a.sptr[sl + 1]) - base) / WAVE;
        const int so = i == 0 ? so0 : a.sofs[sl];
        const int r = sl * WAVE + lane;
        T sum;
        if (NT && base >= a.resident)
            sum = slab_row<T, COLS, true>(a, so, base, lane, r, width);
        else
            sum = slab_row<T, COLS, false>(a, so, base, lane, r, width);
        if (r < a.n) row_epilogue<T, MODE>(a, r, sum, acc[i / 2]);
    }
    if constexpr (MODE != ROW_PLAIN) {
        const int ngroups = a.slabs_per_block / kSlabGroup;
        const int nb = (a.nslabs + kSlabGroup - 1) / kSlabGroup;
        const int g0 = s0 / kSlabGroup;
        const int ng = min(ngroups, nb - g0);
        if constexpr (MODE == ROW_DOT) {
            double v[kMaxGroups][1] = {{acc[0][0]}, {acc[1][0]}};
            store_group_partials<1>(v, ng, a.partials, g0, nb);
        } else {
            store_group_partials<3>(acc, ng, a.partials, g0, nb);
        }
    }
}

// MB: the resident workgroups per CU the kernel is compiled for (launch bound).  1 leaves
// the register budget to the compiler (FP64 products: 84-98 VGPRs, 4-5 wavefronts per SIMD);
// kSellMinBlocks (6) caps it at 80 VGPRs, so 6 wavefronts per SIMD with fewer loads in
// flight in each (no spills in any variant).  Which one is faster depends on the layout
// (more resident wavefronts pay on some orderings and lose on others), so the autotuner
// picks per matrix; both give the same bits.
template <typename T, int MODE, bool DELTA, int MB>
__global__ __launch_bounds__(WG, MB) void k_sell(RowArgs<T> a) {
    // DELTA: the layout's slabs read 16-bit offsets (else 32-bit columns)
    sell_rows<T, MODE, DELTA ? 1 : 0, false>(a);
}

// Layouts with both kinds of per-slot columns.
template <typename T, int MODE, int MB>
__global__ __launch_bounds__(WG, MB) void k_sell_wide(RowArgs<T> a) {
    sell_rows<T, MODE, 2, false>(a);
}

// The same with the matrix values read by nontemporal loads past the first `resident`
// value slots (chosen by the autotuner): the prefix can stay in the Infinity Cache from one
// product to the next while the rest streams past it.
template <typename T, int MODE, bool DELTA, int MB>
__global__ __launch_bounds__(WG, MB) void k_sell_nt(RowArgs<T> a) {
    sell_rows<T, MODE, DELTA ? 1 : 0, true>(a);
}

template <typename T, int MODE, int MB>
__global__ __launch_bounds__(WG, MB) void k_sell_wide_nt(RowArgs<T> a) {
    sell_rows<T, MODE, 2, true>(a);
}

// [row-kernels-end]

// Totals of a START / RESID row kernel -> solver scalars (thread 0 of sample s's block).
template <int MODE>
__device__ void finish_rows(PcgState* st, const double (&tot)[3], int outer_mode) {
    if constexpr (MODE == ROW_START) {
        st->rzs[0] = tot[0];
        st->rzs[1] = 0.0;
        st->rr = tot[1];
        st->bb = tot[2];
        st->rr_first = tot[1];
        st->tol2 = st->tol * st->tol * tot[2];
        st->iters = 0;
        if (st->bad_diag || !finite(tot[0]) || !finite(tot[1]) || !finite(tot[2])) {
            st->status = RAFEM_E_BREAKDOWN;
            st->done = 1;
        } else if (tot[1] <= st->tol2) {
            st->status = RAFEM_OK;
            st->done = 1;
        } else {
            st->status = RAFEM_E_NOCONV;
            st->done = 0;
        }
    } else {  // ROW_RESID
        st->rr = tot[1];
        st->bb = tot[2];
        if (outer_mode) {
            st->tol2 = st->tol * st->tol * tot[2];
            if (st->iters == 0) st->rr_first = tot[1];
            if (st->bad_diag || !finite(tot[1]) || !finite(tot[2])) {
                st->status = RAFEM_E_BREAKDOWN;
                st->done = 1;
            } else if (tot[1] <= st->tol2) {
                st->status = RAFEM_OK;
                st->done = 1;
            } else if (st->iters >= st->maxit) {
                st->status = RAFEM_E_NOCONV;
                st->done = 1;
            } else {
                st->scale_prev = st->scale;
                st->scale = 1.0 / sqrt(tot[1]);
                st->iters += 1;
            }
        }
    }
}

// One block per sample.
template <int MODE>
__global__ __launch_bounds__(WG) void k_finalize_rows(const double* __restrict__ partials, int nb,
                                                      int rpb, PcgState* st, int outer_mode,
                                                      Samples smp) {
    const int s = blockIdx.x;
    if (MODE == ROW_RESID && outer_mode && st[s].done) return;
    int b0, b1;
    sample_blocks(smp, s, rpb, b0, b1);
    double tot[3];
    range_totals<3>(partials, nb, b0, b1, tot);
    if (threadIdx.x == 0) finish_rows<MODE>(st + s, tot, outer_mode);
}

// ---------------------------------------------------------------------------
// Vector kernels (kVecRowsPerBlock rows per workgroup, VPT per thread)
// ---------------------------------------------------------------------------
constexpr int VPT = kVecRowsPerBlock / WG;

// x += alpha p; z -= alpha D^-1 q, alpha = rz / (sample's total of p.Ap); partials of r.z,
// r.r with r = D z.  The recurrence is carried on the preconditioned residual z = D^-1 r
// (the same iterates as the one on r, in exact arithmetic), so that the direction update
// reads z and p only.
template <typename T>
__global__ __launch_bounds__(WG) void k_update(int n, T* __restrict__ x, T* __restrict__ z,
                                               const T* __restrict__ p,
                                               const T* __restrict__ q,
                                               const T* __restrict__ dinv,
                                               const double* __restrict__ pq_part, int nb_pq,
                                               int rpb_pq, const double* __restrict__ pq_tot,
                                               double* __restrict__ rz_part,
                                               const int* __restrict__ itb, int j,
                                               PcgState* st, Samples smp) {
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int row0 = blk * kVecRowsPerBlock;
    const int s = sample_of(smp, row0);
    PcgState& S = st[s];
    // In a batch, finished samples skip their rows before loading them.  A single solve
    // issues its loads first so that they overlap the read of the state (only launches
    // enqueued past convergence waste them).
    if (smp.S > 1 && S.done) return;
    const int it = *itb + j;
    const int i0 = row0 + threadIdx.x;
    T xv[VPT], zv[VPT], pv[VPT], qv[VPT], dv[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) {
            xv[u] = x[i];
            zv[u] = z[i];
            pv[u] = p[i];
            qv[u] = q[i];
            dv[u] = dinv[i];
        }
    }
    // the sample's total of p.Ap: summed by k_sum_partials (many slots), or here
    int b0 = 0, b1 = 0;
    RangeBatch<1> first;
    double pq[1];
    if (pq_tot) {
        pq[0] = pq_tot[s];
    } else {
        sample_blocks(smp, s, rpb_pq, b0, b1);
        range_prefetch<1>(pq_part, nb_pq, b0, b1, first);
    }
    if (S.done) return;
    if (!pq_tot) range_totals<1>(pq_part, nb_pq, b0, b1, pq, &first);
    const bool writer = threadIdx.x == 0 && blk == smp.row_off[s] / kVecRowsPerBlock;
    if (!(pq[0] > 0.0) || !finite(pq[0])) {
        if (writer) {
            S.pq = pq[0];
            S.iters = it;
            S.status = RAFEM_E_BREAKDOWN;
            S.done = 1;
        }
        return;
    }
    const T alpha = (T)(S.rzs[it & 1] / pq[0]);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) {
            const T xi = xv[u] + alpha * pv[u];
            const T zi = zv[u] - alpha * (dv[u] * qv[u]);
            x[i] = xi;
            z[i] = zi;
            // r = z / D^-1 for the two dot products: an FP32 reciprocal (1 ulp) in the
            // FP32 inner solve, whose scalars carry FP32 rounding anyway; exact in FP64
            const double zd = (double)zi;
            double ri;
            if constexpr (sizeof(T) == 4) ri = (double)(zi * __builtin_amdgcn_rcpf(dv[u]));
            else ri = zd / (double)dv[u];
            acc[0] += ri * zd;
            acc[1] += ri * ri;
        }
    }
    store_partials<2>(acc, rz_part, blk, nb);
    if (writer) S.pq = pq[0];
}

// Convergence test on the sample's totals of r.z and r.r, then p = z + beta p.
template <typename T>
__global__ __launch_bounds__(WG) void k_pupdate(int n, T* __restrict__ p,
                                                const T* __restrict__ z,
                                                const double* __restrict__ rz_part, int nb_rz,
                                                const double* __restrict__ rz_tot,
                                                const int* __restrict__ itb, int j, PcgState* st,
                                                Samples smp) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int row0 = blk * kVecRowsPerBlock;
    const int s = sample_of(smp, row0);
    PcgState& S = st[s];
    if (smp.S > 1 && S.done) return;  // as in k_update
    const int it = *itb + j;
    const int i0 = row0 + threadIdx.x;
    T zv[VPT], pv[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) {
            zv[u] = z[i];
            pv[u] = p[i];
        }
    }
    int b0, b1;
    sample_blocks(smp, s, kVecRowsPerBlock, b0, b1);
    RangeBatch<2> first;
    double tot[2];
    if (rz_tot) {
        tot[0] = rz_tot[2 * s];
        tot[1] = rz_tot[2 * s + 1];
    } else {
        range_prefetch<2>(rz_part, nb_rz, b0, b1, first);
    }
    if (S.done) return;
    if (!rz_tot) range_totals<2>(rz_part, nb_rz, b0, b1, tot, &first);
    const double rz = tot[0], rr = tot[1];
    const int iters = it + 1;
    int status = -1;
    if (!finite(rz) || !finite(rr) || rz < 0.0) status = RAFEM_E_BREAKDOWN;
    else if (rr <= S.tol2) status = RAFEM_OK;
    else if (iters >= S.maxit) status = RAFEM_E_NOCONV;
    const bool writer = threadIdx.x == 0 && blk == b0;
    if (status >= 0) {
        if (writer) {
            S.rr = rr;
            S.iters = iters;
            S.status = status;
            S.done = 1;
        }
        return;
    }
    const double beta = rz / S.rzs[it & 1];
    const T bt = (T)beta;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) p[i] = zv[u] + bt * pv[u];
    }
    if (writer) {
        S.rzs[(it + 1) & 1] = rz;
        S.rr = rr;
        S.beta = beta;
        S.iters = iters;
    }
}

// One block per sample: the sample's totals of K partial arrays (range_totals, the same
// slots in the same order as the vector kernels would add them, so the totals are bitwise
// theirs), for a next kernel whose every block would otherwise read all the slots.
template <int K>
__global__ __launch_bounds__(WG) void k_sum_partials(const double* __restrict__ partials, int nb,
                                                     int rpb, Samples smp,
                                                     double* __restrict__ out) {
    const int s = blockIdx.x;
    int b0, b1;
    sample_blocks(smp, s, rpb, b0, b1);
    double tot[K];
    range_totals<K>(partials, nb, b0, b1, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[K * s + k] = tot[k];
    }
}

// Mixed refinement: inner right-hand side r32 = r64 / ||r64||, d32 = 0 and, on a fresh
// start, p32 = D^-1 r32, for the samples whose refinement is not finished.  A continuation
// leaves p32 to k_inner_pcont.
__global__ __launch_bounds__(WG) void k_inner_start(int n, const double* __restrict__ r64,
                                                    const PcgState* outer,
                                                    float* __restrict__ r32,
                                                    float* __restrict__ d32,
                                                    float* __restrict__ p32,
                                                    const float* __restrict__ dinv32,
                                                    double* partials, Samples smp, int cont) {
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int row0 = blk * kVecRowsPerBlock;
    const int s = sample_of(smp, row0);
    const bool skip = outer[s].done != 0;
    const double scale = outer[s].scale;
    const int i0 = row0 + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (!skip) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int i = i0 + u * WG;
            if (i < n) {
                const float ri = (float)(r64[i] * scale);
                const float zi = dinv32[i] * ri;
                r32[i] = zi;  // the inner PCG carries z = D^-1 r
                d32[i] = 0.0f;
                if (!cont) p32[i] = zi;
                acc[0] += (double)ri * (double)zi;
                acc[1] += (double)ri * (double)ri;
            }
        }
    }
    store_partials<2>(acc, partials, blk, nb);
}

// One block per sample: totals of k_inner_start's partials -> inner solver state.  On a
// continuation the state still holds the finished inner solve: its last iteration it =
// iters - 1 kept (r, z) of that iteration in rzs[it & 1], and the new direction's
// coefficient is that recurrence step's beta taken with the new residual,
// rz_new / rz_old, times scale_prev / scale (rz_old was formed at the old scale, and p32
// is carried over to the new one).
__global__ __launch_bounds__(WG) void k_finalize_inner(const double* __restrict__ partials, int nb,
                                                       const PcgState* outer, double inner_tol,
                                                       int maxit, PcgState* inner, Samples smp,
                                                       int cont) {
    const int s = blockIdx.x;
    int b0, b1;
    sample_blocks(smp, s, kVecRowsPerBlock, b0, b1);
    double tot[2];
    range_totals<2>(partials, nb, b0, b1, tot);
    if (threadIdx.x != 0) return;
    PcgState& S = inner[s];
    const bool skip = outer[s].done != 0;
    // the inner solve need not reduce its residual further than a tenth of what the FP64
    // test still asks for (tol ||b|| / ||r||): the last refinement stops there
    double tol_in = inner_tol;
    if (!skip && outer[s].rr > 0.0) tol_in = fmax(inner_tol, 0.1 * sqrt(outer[s].tol2 / outer[s].rr));
    double beta = 0.0;
    if (cont && !skip) {
        const int last = S.iters > 0 ? S.iters - 1 : 0;
        const double rz_old = S.rzs[last & 1];
        beta = (rz_old > 0.0 && finite(rz_old))
                   ? tot[0] / rz_old * (outer[s].scale_prev / outer[s].scale) : 0.0;
    }
    S.rzs[0] = tot[0];
    S.rzs[1] = 0.0;
    S.beta = beta;
    S.rr = tot[1];
    S.bb = tot[1];
    S.rr_first = tot[1];
    S.tol = tol_in;
    S.tol2 = tol_in * tol_in * tot[1];
    S.iters = 0;
    S.maxit = maxit;
    S.bad_diag = 0;
    if (skip || !(tot[1] > 0.0)) {
        S.status = RAFEM_OK;
        S.done = 1;
    } else if (!finite(tot[0]) || !finite(tot[1]) || !finite(beta)) {
        S.status = RAFEM_E_BREAKDOWN;
        S.done = 1;
    } else {
        S.status = RAFEM_E_NOCONV;
        S.done = 0;
    }
}

// Continuation of the inner recurrence: p32 = z32 + beta p32 (z32 = D^-1 r32 as
// k_inner_start left it, beta from k_finalize_inner), for the samples whose inner solve
// goes on.
__global__ __launch_bounds__(WG) void k_inner_pcont(int n, const float* __restrict__ z32,
                                                    float* __restrict__ p32,
                                                    const PcgState* inner, Samples smp) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int row0 = blk * kVecRowsPerBlock;
    const int s = sample_of(smp, row0);
    if (inner[s].done) return;
    const float bt = (float)inner[s].beta;
    const int i0 = row0 + threadIdx.x;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) p32[i] = z32[i] + bt * p32[i];
    }
}

__global__ __launch_bounds__(WG) void k_refine_update(int n, double* __restrict__ x,
                                                      const float* __restrict__ d32,
                                                      const PcgState* outer, Samples smp) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int row0 = blk * kVecRowsPerBlock;
    const int s = sample_of(smp, row0);
    if (outer[s].done) return;
    const double norm = 1.0 / outer[s].scale;
    const int i0 = row0 + threadIdx.x;
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int i = i0 + u * WG;
        if (i < n) x[i] += (double)d32[i] * norm;
    }
}

// The report of a solve enqueued without host synchronisation (one sample): cleared first,
// the inner iterations of each refinement added after it, completed from the final state
// (the solve's, or the refinement's) and the true residual of the returned x.
__global__ void k_info_begin(rafem_device_info* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        info->status = RAFEM_E_NOCONV;
        info->iters = 0;
        info->outer = 0;
        info->pad = 0;
        info->relres_true = 0.0;
    }
}

__global__ void k_info_add_inner(const PcgState* inner, rafem_device_info* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) info->iters += inner->iters;
}

__global__ void k_info_finish(const PcgState* st, const PcgState* chk, int mixed,
                              rafem_device_info* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    info->status = st->done ? st->status : RAFEM_E_NOCONV;
    if (mixed) info->outer = st->iters;
    else info->iters = st->iters;
    const double bb = chk->bb;
    info->relres_true = bb > 0.0 ? sqrt(chk->rr / bb) : sqrt(chk->rr);
}

inline int grid1(int64_t n) { return (int)((n + WG - 1) / WG); }
inline int vec_blocks(int n) { return (n + kVecRowsPerBlock - 1) / kVecRowsPerBlock; }

// A launch, optionally with events stamped when the kernel itself starts and ends (the
// measurement mode: the events then time the kernel alone, not the gap before it).
template <typename K, typename A>
void launch_timed(K kernel, int nb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, const A& a) {
    if (ev0)
        hipExtLaunchKernelGGL(kernel, dim3(nb), dim3(WG), 0, s, ev0, ev1, 0, a);
    else
        hipLaunchKernelGGL(kernel, dim3(nb), dim3(WG), 0, s, a);
}

template <typename T, int MODE>
void launch_csr_kernel(int lanes, int nb, const RowArgs<T>& a, hipStream_t s, hipEvent_t ev0,
                       hipEvent_t ev1) {
    switch (lanes) {
        case 2: launch_timed(k_csr<T, 2, MODE>, nb, s, ev0, ev1, a); break;
        case 8: launch_timed(k_csr<T, 8, MODE>, nb, s, ev0, ev1, a); break;
        case 16: launch_timed(k_csr<T, 16, MODE>, nb, s, ev0, ev1, a); break;
        default: launch_timed(k_csr<T, 4, MODE>, nb, s, ev0, ev1, a); break;
    }
}

// The slab kernel for this layout's column kinds and the configured value loads.
template <typename T, int MODE, int MB>
void (*sell_kernel(const Mat& A, int stream))(RowArgs<T>) {
    if (A.sdel && A.wide) return stream ? k_sell_wide_nt<T, MODE, MB> : k_sell_wide<T, MODE, MB>;
    if (A.sdel) return stream ? k_sell_nt<T, MODE, true, MB> : k_sell<T, MODE, true, MB>;
    return stream ? k_sell_nt<T, MODE, false, MB> : k_sell<T, MODE, false, MB>;
}

// One launcher for both layouts.  Returns {grid size, rows per block}.
template <typename T, int MODE>
GridInfo launch_rows(const Mat& A, const T* vals, const SpmvConfig& c, const T* x, T* y,
                     const double* b, const double* dinv, double* pout, double* partials,
                     PcgState* st, const Samples& smp, int outer_mode, hipStream_t s,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    RowArgs<T> a{A.rp,   A.ci, A.sptr, A.scol,   A.sdel, A.sofs, A.soff,
                 vals,   x,    y,      b,        dinv,   pout,   partials,
                 st,     smp,  A.n,    A.nslabs, c.rows_per_block, c.slabs_per_block,
                 outer_mode, c.resident};
    GridInfo g;
    if (A.sell) {
        const int nblk = blocks_for(A.nslabs, c.slabs_per_block);
        g.nb = blocks_for(A.nslabs, kSlabGroup);  // partial slots: one per group of slabs
        g.rpb = kSlabGroup * WAVE;
        if (nblk > 0) {
            void (*k)(RowArgs<T>) = c.min_blocks == kSellMinBlocks
                                        ? sell_kernel<T, MODE, kSellMinBlocks>(A, c.stream)
                                        : sell_kernel<T, MODE, 1>(A, c.stream);
            launch_timed(k, nblk, s, ev0, ev1, a);
        }
    } else {
        g.nb = blocks_for(A.n, c.rows_per_block);
        g.rpb = c.rows_per_block;
        if (g.nb > 0) launch_csr_kernel<T, MODE>(c.lanes, g.nb, a, s, ev0, ev1);
    }
    return g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int blocks_for(int64_t n, int rows_per_block) {
    return (int)((n + rows_per_block - 1) / rows_per_block);
}

SpmvConfig choose_spmv_config(int64_t n, int64_t nnz) {
    const double avg = n > 0 ? (double)nnz / (double)n : 1.0;
    SpmvConfig c;
    c.lanes = avg > 6.0 ? 4 : 2;
    const int rows_per_pass = WG / c.lanes;
    int passes = 8;
    // keep at least ~4 blocks per CU when the matrix is small
    while (passes > 1 && blocks_for(n, rows_per_pass * passes) < 1024) passes /= 2;
    c.rows_per_block = rows_per_pass * passes;
    // two slabs per wavefront: one group of partial sums per workgroup (the autotuner may
    // move to two groups)
    c.slabs_per_block = kSlabGroup;
    return c;
}

void launch_state_init(PcgState* st, int S, double tol, int maxit, int* itb, hipStream_t s) {
    const int grid = S > 0 ? (S + 63) / 64 : 1;
    hipLaunchKernelGGL(k_state_init, dim3(grid), dim3(64), 0, s, st, S, tol, maxit, itb);
}

void launch_advance(int* itb, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, itb, k);
}

void launch_diag_inv(const Mat& A, double* dinv, float* dinv32, PcgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_inv, dim3(grid1(A.n)), dim3(WG), 0, s, A.rp, A.ci, A.v, A.n, dinv,
                       dinv32, st);
}

void launch_pcg_start(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                      const double* dinv, double* r, double* p, double* partials, PcgState* st,
                      const Samples& smp, hipStream_t s) {
    const GridInfo g = launch_rows<double, ROW_START>(A, A.v, c, x, r, b, dinv, p, partials, st,
                                                      smp, 0, s);
    hipLaunchKernelGGL(k_finalize_rows<ROW_START>, dim3(smp.S), dim3(WG), 0, s, partials, g.nb,
                       g.rpb, st, 0, smp);
}

GridInfo launch_spmv_dot64(const Mat& A, const SpmvConfig& c, const double* p, double* q,
                           double* pq_part, PcgState* st, const Samples& smp, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
    return launch_rows<double, ROW_DOT>(A, A.v, c, p, q, nullptr, nullptr, nullptr, pq_part, st,
                                        smp, 0, s, ev0, ev1);
}

GridInfo launch_spmv_dot32(const Mat& A, const SpmvConfig& c, const float* p, float* q,
                           double* pq_part, PcgState* st, const Samples& smp, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
    return launch_rows<float, ROW_DOT>(A, A.v32, c, p, q, nullptr, nullptr, nullptr, pq_part, st,
                                       smp, 0, s, ev0, ev1);
}

void launch_spmv64(const Mat& A, const SpmvConfig& c, const double* x, double* y,
                   hipStream_t s) {
    Samples one{1, nullptr};
    launch_rows<double, ROW_PLAIN>(A, A.v, c, x, y, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   one, 0, s);
}

void launch_spmv32(const Mat& A, const SpmvConfig& c, const float* x, float* y,
                   hipStream_t s) {
    Samples one{1, nullptr};
    launch_rows<float, ROW_PLAIN>(A, A.v32, c, x, y, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  one, 0, s);
}

void launch_residual64(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                       double* r, double* partials, PcgState* st, const Samples& smp,
                       int outer_mode, hipStream_t s) {
    const GridInfo g = launch_rows<double, ROW_RESID>(A, A.v, c, x, r, b, nullptr, nullptr,
                                                      partials, st, smp, outer_mode, s);
    hipLaunchKernelGGL(k_finalize_rows<ROW_RESID>, dim3(smp.S), dim3(WG), 0, s, partials, g.nb,
                       g.rpb, st, outer_mode, smp);
}

// The sample totals a vector kernel needs, pre-summed by one block per sample when a
// sample has more than kDirectSlots partial slots (else every block adds them itself: one
// kernel fewer).  Returns the totals' array, or NULL for the direct form.
constexpr int kDirectSlots = 2500;

template <int K>
const double* presum(const double* partials, int nb, int rpb, const Samples& smp, double* sums,
                     hipStream_t s) {
    if (!sums || smp.max_rows <= 0 || (smp.max_rows + rpb - 1) / rpb <= kDirectSlots)
        return nullptr;
    hipLaunchKernelGGL(k_sum_partials<K>, dim3(smp.S), dim3(WG), 0, s, partials, nb, rpb, smp,
                       sums);
    return sums;
}

int launch_update64(int n, double* x, double* r, const double* p, const double* q,
                    const double* dinv, const double* pq_part, const GridInfo& gpq,
                    double* rz_part, const int* itb, int j, PcgState* st, const Samples& smp,
                    double* sums, hipStream_t s) {
    const int nb = vec_blocks(n);
    const double* tot = presum<1>(pq_part, gpq.nb, gpq.rpb, smp, sums, s);
    hipLaunchKernelGGL(k_update<double>, dim3(nb), dim3(WG), 0, s, n, x, r, p, q, dinv, pq_part,
                       gpq.nb, gpq.rpb, tot, rz_part, itb, j, st, smp);
    return nb;
}

int launch_update32(int n, float* x, float* r, const float* p, const float* q, const float* dinv,
                    const double* pq_part, const GridInfo& gpq, double* rz_part, const int* itb,
                    int j, PcgState* st, const Samples& smp, double* sums, hipStream_t s) {
    const int nb = vec_blocks(n);
    const double* tot = presum<1>(pq_part, gpq.nb, gpq.rpb, smp, sums, s);
    hipLaunchKernelGGL(k_update<float>, dim3(nb), dim3(WG), 0, s, n, x, r, p, q, dinv, pq_part,
                       gpq.nb, gpq.rpb, tot, rz_part, itb, j, st, smp);
    return nb;
}

void launch_pupdate64(int n, double* p, const double* z, const double* rz_part, int nb_rz,
                      const int* itb, int j, PcgState* st, const Samples& smp, double* sums,
                      hipStream_t s) {
    const double* tot =
        presum<2>(rz_part, nb_rz, kVecRowsPerBlock, smp, sums ? sums + smp.S : nullptr, s);
    hipLaunchKernelGGL(k_pupdate<double>, dim3(vec_blocks(n)), dim3(WG), 0, s, n, p, z, rz_part,
                       nb_rz, tot, itb, j, st, smp);
}

void launch_pupdate32(int n, float* p, const float* z, const double* rz_part, int nb_rz,
                      const int* itb, int j, PcgState* st, const Samples& smp, double* sums,
                      hipStream_t s) {
    const double* tot =
        presum<2>(rz_part, nb_rz, kVecRowsPerBlock, smp, sums ? sums + smp.S : nullptr, s);
    hipLaunchKernelGGL(k_pupdate<float>, dim3(vec_blocks(n)), dim3(WG), 0, s, n, p, z, rz_part,
                       nb_rz, tot, itb, j, st, smp);
}

void launch_inner_start(int n, const double* r64, const PcgState* outer, float* r32, float* d32,
                        float* p32, const float* dinv32, double inner_tol, int maxit,
                        double* partials, PcgState* inner, const Samples& smp, int cont,
                        hipStream_t s) {
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_inner_start, dim3(nb), dim3(WG), 0, s, n, r64, outer, r32, d32, p32,
                       dinv32, partials, smp, cont);
    hipLaunchKernelGGL(k_finalize_inner, dim3(smp.S), dim3(WG), 0, s, partials, nb, outer,
                       inner_tol, maxit, inner, smp, cont);
    if (cont)
        hipLaunchKernelGGL(k_inner_pcont, dim3(nb), dim3(WG), 0, s, n, r32, p32, inner, smp);
}

void launch_refine_update(int n, double* x, const float* d32, const PcgState* outer,
                          const Samples& smp, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_update, dim3(vec_blocks(n)), dim3(WG), 0, s, n, x, d32, outer,
                       smp);
}

void launch_info_begin(rafem_device_info* info, hipStream_t s) {
    hipLaunchKernelGGL(k_info_begin, dim3(1), dim3(64), 0, s, info);
}

void launch_info_add_inner(const PcgState* inner, rafem_device_info* info, hipStream_t s) {
    hipLaunchKernelGGL(k_info_add_inner, dim3(1), dim3(64), 0, s, inner, info);
}

void launch_info_finish(const PcgState* st, const PcgState* chk, int mixed,
                        rafem_device_info* info, hipStream_t s) {
    hipLaunchKernelGGL(k_info_finish, dim3(1), dim3(64), 0, s, st, chk, mixed, info);
}

}  // namespace rafem
