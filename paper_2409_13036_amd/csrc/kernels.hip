// HIP kernels for gfx950 (CDNA4, wave64): Jacobi-PCG building blocks and
// element-parallel, colour-by-colour FEM assembly.
//
// Everything here is HBM-bound (sparse matrix-vector products and vector
// updates at ~0.1-0.2 flop/byte), so the kernels are organised for coalesced
// streaming and few passes over memory, not for matrix cores:
//   * row kernels: a group of LANES consecutive lanes owns one CSR row, so a
//     wave streams a contiguous range of values/column indices; the group sum
//     is a wave shuffle; dot products are fused into the same pass;
//   * workgroups own contiguous row ranges and are remapped so each of the 8
//     XCDs (own L2) walks one contiguous eighth of the rows, which keeps the
//     x-gathers of neighbouring rows in that XCD's L2;
//   * reductions are deterministic and need no atomics or fences: each block
//     stores its partial sums in a fixed slot, and the consumer (every block of
//     the next kernel, or a one-block finalize kernel) adds them in index order
//     after the kernel boundary; solver scalars stay in device memory, so there
//     is no host round trip per iteration.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fem_device.hpp"
#include "internal.hpp"

namespace rafem {
namespace {

using namespace dev;


// ---------------------------------------------------------------------------
// Solver state
// ---------------------------------------------------------------------------
__global__ void k_state_init(PcgState* st, double tol, int maxit) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rzs[0] = st->rzs[1] = st->pq = st->beta = st->rr = st->bb = 0.0;
        st->tol = tol;
        st->tol2 = 0.0;
        st->scale = 1.0;
        st->rr_first = 0.0;
        st->iters = 0;
        st->maxit = maxit;
        st->done = 0;
        st->status = RAFEM_E_NOCONV;
        st->bad_diag = 0;
    }
}

// dinv = 1 / diag(A) (also as FP32).  A missing or non-positive diagonal marks the state.
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
// Row kernels (CSR, LANES lanes per row)
// ---------------------------------------------------------------------------
enum RowMode : int {
    ROW_PLAIN = 0,  // y = A x
    ROW_DOT = 1,    // y = A x, sum x.y -> alpha (PCG step; early exit when done)
    ROW_START = 2,  // y = b - A x, p = D^-1 y, sums y.p, y.y, b.b (PCG start)
    ROW_RESID = 3,  // y = b - A x, sums y.y, b.b (refinement residual / true residual)
};

template <typename T>
struct RowArgs {
    const int* __restrict__ rp;
    const int* __restrict__ ci;
    const T* __restrict__ val;
    const T* __restrict__ x;
    T* __restrict__ y;
    const double* __restrict__ b;
    const double* __restrict__ dinv;
    double* __restrict__ pout;
    double* partials;
    PcgState* st;
    int n;
    int rows_per_block;
    int outer_mode;
};

// Thread 0 of the last block: turn the grid totals of a row kernel into solver scalars.
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
                st->scale = 1.0 / sqrt(tot[1]);
                st->iters += 1;
            }
        }
    }
}

template <typename T, int LANES, int MODE>
__global__ __launch_bounds__(WG) void k_rows(RowArgs<T> a) {
    if constexpr (MODE == ROW_DOT) {
        if (a.st->done) return;
    }
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int row0 = blk * a.rows_per_block;
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
        if (sub == 0) {
            if constexpr (MODE == ROW_PLAIN) {
                a.y[r] = sum;
            } else if constexpr (MODE == ROW_DOT) {
                a.y[r] = sum;
                acc[0] += (double)a.x[r] * (double)sum;
            } else {
                const double bi = a.b[r];
                const double ri = bi - (double)sum;
                a.y[r] = (T)ri;
                acc[1] += ri * ri;
                acc[2] += bi * bi;
                if constexpr (MODE == ROW_START) {
                    const double zi = a.dinv[r] * ri;
                    a.pout[r] = zi;
                    acc[0] += ri * zi;
                }
            }
        }
    }
    if constexpr (MODE == ROW_PLAIN) {
        return;
    } else if constexpr (MODE == ROW_DOT) {
        double v1[1] = {acc[0]};
        store_partials<1>(v1, a.partials, blk, nb);
    } else {
        store_partials<3>(acc, a.partials, blk, nb);
    }
}

// ---------------------------------------------------------------------------
// SELL kernels: 64-row slabs, one row per lane.  Entry j of the 64 rows of a slab is
// one contiguous 64-word load for values and for column ids; for the banded meshes
// here the x-gathers of a slab are contiguous too.  Rows are summed in entry order.
// ---------------------------------------------------------------------------
template <typename T>
struct SellArgs {
    const int* __restrict__ sptr;
    const int* __restrict__ scol;     // absolute column ids (used when sdel is NULL)
    const int16_t* __restrict__ sdel; // column - row offsets
    const T* __restrict__ val;
    const T* __restrict__ x;
    T* __restrict__ y;
    const double* __restrict__ b;
    const double* __restrict__ dinv;
    double* __restrict__ pout;
    double* partials;
    PcgState* st;
    int n;
    int nslabs;
    int slabs_per_block;
    int outer_mode;
};

constexpr int kSellUnroll = 9;

// Sum over the entries of one row in entry order.  COL is int (absolute columns, xr = x)
// or int16_t (offsets to the row, xr = x + row).
template <typename T, typename COL>
__device__ __forceinline__ T sell_row(const COL* __restrict__ cp, const T* __restrict__ vp,
                                      const T* __restrict__ xr, int width) {
    T sum = T(0);
    int j = 0;
    for (; j + kSellUnroll <= width; j += kSellUnroll) {
        int c[kSellUnroll];
        T v[kSellUnroll];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) {
            c[u] = cp[(j + u) * WAVE];
            v[u] = vp[(j + u) * WAVE];
        }
        T g[kSellUnroll];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) g[u] = xr[c[u]];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) sum += v[u] * g[u];
    }
    for (; j < width; ++j) sum += vp[j * WAVE] * xr[cp[j * WAVE]];
    return sum;
}

template <typename T, int MODE, bool DELTA>
__global__ __launch_bounds__(WG) void k_sell(SellArgs<T> a) {
    if constexpr (MODE == ROW_DOT) {
        if (a.st->done) return;
    }
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int s0 = blk * a.slabs_per_block;
    const int s1 = min(s0 + a.slabs_per_block, a.nslabs);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int sl = s0 + w; sl < s1; sl += NWAVES) {
        const int base = a.sptr[sl];
        const int width = (a.sptr[sl + 1] - base) / WAVE;
        const int r = sl * WAVE + lane;
        T sum;
        if constexpr (DELTA)
            sum = sell_row<T, int16_t>(a.sdel + base + lane, a.val + base + lane,
                                       a.x + min(r, a.n - 1), width);
        else
            sum = sell_row<T, int>(a.scol + base + lane, a.val + base + lane, a.x, width);
        if (r < a.n) {
            if constexpr (MODE == ROW_PLAIN) {
                a.y[r] = sum;
            } else if constexpr (MODE == ROW_DOT) {
                a.y[r] = sum;
                acc[0] += (double)a.x[r] * (double)sum;
            } else {
                const double bi = a.b[r];
                const double ri = bi - (double)sum;
                a.y[r] = (T)ri;
                acc[1] += ri * ri;
                acc[2] += bi * bi;
                if constexpr (MODE == ROW_START) {
                    const double zi = a.dinv[r] * ri;
                    a.pout[r] = zi;
                    acc[0] += ri * zi;
                }
            }
        }
    }
    if constexpr (MODE == ROW_PLAIN) {
        return;
    } else if constexpr (MODE == ROW_DOT) {
        double v1[1] = {acc[0]};
        store_partials<1>(v1, a.partials, blk, nb);
    } else {
        store_partials<3>(acc, a.partials, blk, nb);
    }
}

// One block: totals of a START / RESID row kernel's partials -> solver scalars.
template <int MODE>
__global__ __launch_bounds__(WG) void k_finalize_rows(const double* __restrict__ partials, int nb,
                                                      PcgState* st, int outer_mode) {
    double tot[3];
    grid_totals<3>(partials, nb, tot);
    if (threadIdx.x == 0) finish_rows<MODE>(st, tot, outer_mode);
}

// ---------------------------------------------------------------------------
// Vector kernels (4 rows per thread, contiguous block ranges)
// ---------------------------------------------------------------------------
constexpr int VPT = kVecRowsPerBlock / WG;

// x += alpha p; r -= alpha q with alpha = rz / sum(p.Ap partials); partials of r.z, r.r.
template <typename T>
__global__ __launch_bounds__(WG) void k_update(int n, T* __restrict__ x, T* __restrict__ r,
                                               const T* __restrict__ p,
                                               const T* __restrict__ q,
                                               const T* __restrict__ dinv,
                                               const double* __restrict__ pq_part, int nb_pq,
                                               double* __restrict__ rz_part, int it,
                                               PcgState* st) {
    if (st->done) return;
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i0 = blk * kVecRowsPerBlock + threadIdx.x;
    // issue this thread's loads before the partial sums so their latency overlaps
    T xv[VPT], rv[VPT], pv[VPT], qv[VPT], dv[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = i0 + j * WG;
        if (i < n) {
            xv[j] = x[i];
            rv[j] = r[i];
            pv[j] = p[i];
            qv[j] = q[i];
            dv[j] = dinv[i];
        }
    }
    double pq[1];
    grid_totals<1>(pq_part, nb_pq, pq);
    if (!(pq[0] > 0.0) || !finite(pq[0])) {
        if (blk == 0 && threadIdx.x == 0) {
            st->pq = pq[0];
            st->iters = it;
            st->status = RAFEM_E_BREAKDOWN;
            st->done = 1;
        }
        return;
    }
    const T alpha = (T)(st->rzs[it & 1] / pq[0]);
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = i0 + j * WG;
        if (i < n) {
            const T xi = xv[j] + alpha * pv[j];
            const T ri = rv[j] - alpha * qv[j];
            x[i] = xi;
            r[i] = ri;
            const T zi = dv[j] * ri;
            acc[0] += (double)ri * (double)zi;
            acc[1] += (double)ri * (double)ri;
        }
    }
    store_partials<2>(acc, rz_part, blk, nb);
    if (blk == 0 && threadIdx.x == 0) st->pq = pq[0];
}

// Convergence test on the totals of r.z and r.r, then p = D^-1 r + beta p.
template <typename T>
__global__ __launch_bounds__(WG) void k_pupdate(int n, T* __restrict__ p,
                                                const T* __restrict__ r,
                                                const T* __restrict__ dinv,
                                                const double* __restrict__ rz_part, int nb_rz,
                                                int it, PcgState* st) {
    if (st->done) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i0 = blk * kVecRowsPerBlock + threadIdx.x;
    T rv[VPT], pv[VPT], dv[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = i0 + j * WG;
        if (i < n) {
            rv[j] = r[i];
            pv[j] = p[i];
            dv[j] = dinv[i];
        }
    }
    double tot[2];
    grid_totals<2>(rz_part, nb_rz, tot);
    const double rz = tot[0], rr = tot[1];
    const int iters = it + 1;
    int status = -1;
    if (!finite(rz) || !finite(rr) || rz < 0.0) status = RAFEM_E_BREAKDOWN;
    else if (rr <= st->tol2) status = RAFEM_OK;
    else if (iters >= st->maxit) status = RAFEM_E_NOCONV;
    const bool writer = blk == 0 && threadIdx.x == 0;
    if (status >= 0) {
        if (writer) {
            st->rr = rr;
            st->iters = iters;
            st->status = status;
            st->done = 1;
        }
        return;
    }
    const double beta = rz / st->rzs[it & 1];
    const T bt = (T)beta;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = i0 + j * WG;
        if (i < n) p[i] = dv[j] * rv[j] + bt * pv[j];
    }
    if (writer) {
        st->rzs[(it + 1) & 1] = rz;
        st->rr = rr;
        st->beta = beta;
        st->iters = iters;
    }
}

// Mixed refinement: inner right-hand side r32 = r64 / ||r64||, d32 = 0, p32 = D^-1 r32.
__global__ __launch_bounds__(WG) void k_inner_start(int n, const double* __restrict__ r64,
                                                    const PcgState* outer,
                                                    float* __restrict__ r32,
                                                    float* __restrict__ d32,
                                                    float* __restrict__ p32,
                                                    const float* __restrict__ dinv32,
                                                    double* partials) {
    const bool skip = outer->done != 0;
    const double scale = outer->scale;
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i0 = blk * kVecRowsPerBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (!skip) {
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            const int i = i0 + j * WG;
            if (i < n) {
                const float ri = (float)(r64[i] * scale);
                const float zi = dinv32[i] * ri;
                r32[i] = ri;
                d32[i] = 0.0f;
                p32[i] = zi;
                acc[0] += (double)ri * (double)zi;
                acc[1] += (double)ri * (double)ri;
            }
        }
    }
    store_partials<2>(acc, partials, blk, nb);
}

// One block: totals of k_inner_start's partials -> inner solver state.
__global__ __launch_bounds__(WG) void k_finalize_inner(const double* __restrict__ partials, int nb,
                                                       const PcgState* outer, double inner_tol,
                                                       int maxit, PcgState* inner) {
    double tot[2];
    grid_totals<2>(partials, nb, tot);
    if (threadIdx.x != 0) return;
    const bool skip = outer->done != 0;
    inner->rzs[0] = tot[0];
    inner->rzs[1] = 0.0;
    inner->rr = tot[1];
    inner->bb = tot[1];
    inner->rr_first = tot[1];
    inner->tol = inner_tol;
    inner->tol2 = inner_tol * inner_tol * tot[1];
    inner->iters = 0;
    inner->maxit = maxit;
    inner->bad_diag = 0;
    if (skip || !(tot[1] > 0.0)) {
        inner->status = RAFEM_OK;
        inner->done = 1;
    } else if (!finite(tot[0]) || !finite(tot[1])) {
        inner->status = RAFEM_E_BREAKDOWN;
        inner->done = 1;
    } else {
        inner->status = RAFEM_E_NOCONV;
        inner->done = 0;
    }
}

__global__ __launch_bounds__(WG) void k_refine_update(int n, double* __restrict__ x,
                                                      const float* __restrict__ d32,
                                                      const PcgState* outer) {
    if (outer->done) return;
    const double norm = 1.0 / outer->scale;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i0 = blk * kVecRowsPerBlock + threadIdx.x;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = i0 + j * WG;
        if (i < n) x[i] += (double)d32[i] * norm;
    }
}

// ---------------------------------------------------------------------------
// Assembly helpers
// ---------------------------------------------------------------------------
__global__ void k_fill(double* __restrict__ v, int64_t n, double value) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) v[i] = value;
}

__global__ void k_cast32(const double* __restrict__ v, float* __restrict__ v32, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) v32[i] = (float)v[i];
}

__global__ void k_coef(const double* __restrict__ perf, double c0, double* __restrict__ coef,
                       int64_t E) {
    const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (e < E) coef[e] = c0 + perf[e];
}

__global__ void k_scatter_dirichlet(const int* __restrict__ ids, const double* __restrict__ vals,
                                    int64_t nD, double* __restrict__ gnode) {
    const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (k < nD) gnode[ids[k]] = vals[k];
}

__global__ void k_set_dirichlet(const int* __restrict__ ids, const double* __restrict__ gnode,
                                int64_t nD, double* __restrict__ x) {
    const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (k < nD) x[ids[k]] = gnode[ids[k]];
}

// One thread per (element of this colour, local row a): add row a of
// mass[e] M_e + stiff[e] K_e into the matrix values.  Elements of one colour share no
// node, so no two threads of a launch touch the same row.  e2s, when given, holds the
// value position of every (element, a, b) pair; otherwise it is searched in the row.
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_assemble(const int* __restrict__ elems, int count,
                                                 const int* __restrict__ conn,
                                                 const double* __restrict__ xyz,
                                                 const Layout L, const int* __restrict__ e2s,
                                                 const double* __restrict__ mass,
                                                 const double* __restrict__ stiff,
                                                 double* __restrict__ vals) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= count * NPE) return;
    const int e = elems[t / NPE];
    const int a = t % NPE;
    int nodes[NPE];
    double X[NPE][3];
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        nodes[b] = conn[(int64_t)e * NPE + b];
#pragma unroll
        for (int i = 0; i < 3; ++i) X[b][i] = xyz[(int64_t)nodes[b] * 3 + i];
    }
    const double m = mass ? mass[e] : 0.0;
    const double c = stiff ? stiff[e] : 0.0;
    double Kr[NPE], Mr[NPE];
    if constexpr (NPE == 8) {
        if constexpr (AFFINE) hex_rows_affine(X, a, Kr, Mr);
        else hex_rows(X, a, Kr, Mr);
    } else {
        double G[4][3];
        const double V = tet_geometry(X, G);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            Kr[b] = V * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
            Mr[b] = (a == b ? 2.0 : 1.0) * V / 20.0;
        }
    }
    if (e2s) {
        const int* sl = e2s + ((int64_t)e * NPE + a) * NPE;
#pragma unroll
        for (int b = 0; b < NPE; ++b) vals[sl[b]] += m * Mr[b] + c * Kr[b];
    } else {
        int start, len, stride;
        row_span(L, nodes[a], start, len, stride);
#pragma unroll
        for (int b = 0; b < NPE; ++b) {
            const int k = find_slot(L.cols, start, len, stride, nodes[b]);
            vals[k] += m * Mr[b] + c * Kr[b];
        }
    }
}

// Value position of every (element, local row a, local column b) in a layout.
__global__ __launch_bounds__(WG) void k_slot_map(int64_t E, int npe, const int* __restrict__ conn,
                                                 const Layout L, int* __restrict__ e2s) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= E * npe) return;
    const int64_t e = t / npe;
    int start, len, stride;
    row_span(L, conn[t], start, len, stride);
    for (int b = 0; b < npe; ++b)
        e2s[t * npe + b] = find_slot(L.cols, start, len, stride, conn[e * npe + b]);
}

// Symmetric lifting of Dirichlet rows/columns, Jacobi inverse and FP32 copy.
__global__ __launch_bounds__(WG) void k_lift(int n, const Layout L, double* __restrict__ vals,
                                             float* __restrict__ vals32,
                                             const uint8_t* __restrict__ isD,
                                             const double* __restrict__ gnode,
                                             double* __restrict__ lift, double* __restrict__ dinv,
                                             float* __restrict__ dinv32, int do_lift) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    int start, len, stride;
    row_span(L, i, start, len, stride);
    double diag = 0.0;
    if (do_lift && isD[i]) {
        for (int j = 0; j < len; ++j) {
            const int k = start + j * stride;
            const double v = (L.cols[k] == i) ? 1.0 : 0.0;
            vals[k] = v;
            if (vals32) vals32[k] = (float)v;
        }
        diag = 1.0;
        if (lift) lift[i] = gnode[i];
    } else {
        double acc = 0.0;
        for (int j = 0; j < len; ++j) {
            const int k = start + j * stride;
            const int c = L.cols[k];
            double v = vals[k];
            if (do_lift && isD[c]) {
                acc += v * gnode[c];
                v = 0.0;
                vals[k] = 0.0;
            }
            if (c == i) diag = v;
            if (vals32) vals32[k] = (float)v;
        }
        if (do_lift && lift) lift[i] = -acc;
    }
    if (dinv) {
        const double inv = 1.0 / diag;
        dinv[i] = inv;
        if (dinv32) dinv32[i] = (float)inv;
    }
}

__global__ __launch_bounds__(WG) void k_sigma(int npe, int64_t E, const int* __restrict__ conn,
                                              const double* __restrict__ T,
                                              const double* __restrict__ sigma0, double alpha,
                                              double T_ref, double* __restrict__ sigma) {
    const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int a = 0; a < npe; ++a) s += T[conn[e * npe + a]];
    sigma[e] = sigma0[e] * (1.0 + alpha * (s / npe - T_ref));
}

// Bioheat right-hand side, one thread per (element of this colour, local node a):
// rhs[node a] += sum_b M_ab (rho_c_dt T_b + perf_e T_a) + int N_a sigma_e |grad V|^2.
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_bioheat_rhs(const int* __restrict__ elems, int count,
                                                    const int* __restrict__ conn,
                                                    const double* __restrict__ xyz,
                                                    const double* __restrict__ T,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ sigma,
                                                    const double* __restrict__ perf,
                                                    double rho_c_dt, double T_a, int with_joule,
                                                    double* __restrict__ rhs) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= count * NPE) return;
    const int e = elems[t / NPE];
    const int a = t % NPE;
    int nodes[NPE];
    double X[NPE][3], Tw[NPE], Vb[NPE];
    const double src = perf[e] * T_a;
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        nodes[b] = conn[(int64_t)e * NPE + b];
#pragma unroll
        for (int i = 0; i < 3; ++i) X[b][i] = xyz[(int64_t)nodes[b] * 3 + i];
        Tw[b] = rho_c_dt * T[nodes[b]] + src;
        Vb[b] = with_joule ? V[nodes[b]] : 0.0;
    }
    const double sg = with_joule ? sigma[e] : 0.0;
    double f = 0.0;
    if constexpr (NPE == 8) {
        double Ji[3][3];
        double det = 0.0;
        if constexpr (AFFINE) det = hex_affine_jacobian(X, Ji);
        for (int q = 0; q < 8; ++q) {
            double xi, et, ze;
            gauss_point(q, xi, et, ze);
            if constexpr (!AFFINE) det = hex_jacobian(X, xi, et, ze, Ji);
            double Nw = 0.0, gv0 = 0.0, gv1 = 0.0, gv2 = 0.0, Na = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                double Nb, d0, d1, d2;
                hex_shape(b, xi, et, ze, Nb, d0, d1, d2);
                if (b == a) Na = Nb;
                Nw += Nb * Tw[b];
                gv0 += Vb[b] * d0;
                gv1 += Vb[b] * d1;
                gv2 += Vb[b] * d2;
            }
            double gV[3];
            grad_x(Ji, gv0, gv1, gv2, gV);
            f += det * Na * (Nw + sg * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]));
        }
    } else {
        double G[4][3];
        const double vol = tet_geometry(X, G);
        double sumw = 0.0, gV[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            sumw += Tw[b];
#pragma unroll
            for (int i = 0; i < 3; ++i) gV[i] += Vb[b] * G[b][i];
        }
        f = vol / 20.0 * (sumw + Tw[a]) +
            sg * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]) * vol / 4.0;
    }
    rhs[nodes[a]] += f;
}

__global__ void k_finish_rhs(int n, const double* __restrict__ rhs,
                             const double* __restrict__ lift, const uint8_t* __restrict__ isD,
                             double* __restrict__ b) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < n) b[i] = isD[i] ? lift[i] : rhs[i] + lift[i];
}

inline int grid1(int64_t n) { return (int)((n + WG - 1) / WG); }

template <typename T, int MODE>
void launch_csr(const SpmvConfig& c, const RowArgs<T>& a, hipStream_t s) {
    const int nb = blocks_for(a.n, c.rows_per_block);
    if (nb == 0) return;
    switch (c.lanes) {
        case 2: hipLaunchKernelGGL((k_rows<T, 2, MODE>), dim3(nb), dim3(WG), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_rows<T, 8, MODE>), dim3(nb), dim3(WG), 0, s, a); break;
        case 16: hipLaunchKernelGGL((k_rows<T, 16, MODE>), dim3(nb), dim3(WG), 0, s, a); break;
        default: hipLaunchKernelGGL((k_rows<T, 4, MODE>), dim3(nb), dim3(WG), 0, s, a); break;
    }
}

// One launcher for both layouts: CSR row groups or SELL slabs.  Returns the grid size.
template <typename T, int MODE>
int launch_rows(const Mat& A, const T* vals, const SpmvConfig& c, const T* x, T* y,
                const double* b, const double* dinv, double* pout, double* partials,
                PcgState* st, int outer_mode, hipStream_t s) {
    if (A.sell) {
        SellArgs<T> a{A.sptr, A.scol, A.sdel, vals, x, y, b, dinv, pout, partials, st, A.n,
                      A.nslabs, c.slabs_per_block, outer_mode};
        const int nb = blocks_for(A.nslabs, c.slabs_per_block);
        if (nb > 0) {
            if (A.sdel)
                hipLaunchKernelGGL((k_sell<T, MODE, true>), dim3(nb), dim3(WG), 0, s, a);
            else
                hipLaunchKernelGGL((k_sell<T, MODE, false>), dim3(nb), dim3(WG), 0, s, a);
        }
        return nb;
    }
    RowArgs<T> a{A.rp, A.ci, vals, x, y, b, dinv, pout, partials, st, A.n, c.rows_per_block,
                 outer_mode};
    launch_csr<T, MODE>(c, a, s);
    return blocks_for(A.n, c.rows_per_block);
}

inline int vec_blocks(int n) { return (n + kVecRowsPerBlock - 1) / kVecRowsPerBlock; }

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
    const int64_t nslabs = (n + WAVE - 1) / WAVE;
    int spw = 2;  // slabs per wavefront
    while (spw > 1 && blocks_for(nslabs, NWAVES * spw) < 1024) spw /= 2;
    c.slabs_per_block = NWAVES * spw;
    return c;
}

void launch_state_init(PcgState* st, double tol, int maxit, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, maxit);
}

void launch_diag_inv(const Mat& A, double* dinv, float* dinv32, PcgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_inv, dim3(grid1(A.n)), dim3(WG), 0, s, A.rp, A.ci, A.v, A.n, dinv,
                       dinv32, st);
}

void launch_pcg_start(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                      const double* dinv, double* r, double* p, double* partials, PcgState* st,
                      hipStream_t s) {
    const int nb = launch_rows<double, ROW_START>(A, A.v, c, x, r, b, dinv, p, partials, st, 0, s);
    hipLaunchKernelGGL(k_finalize_rows<ROW_START>, dim3(1), dim3(WG), 0, s, partials, nb, st, 0);
}

int launch_spmv_dot64(const Mat& A, const SpmvConfig& c, const double* p, double* q,
                      double* pq_part, PcgState* st, hipStream_t s) {
    return launch_rows<double, ROW_DOT>(A, A.v, c, p, q, nullptr, nullptr, nullptr, pq_part, st, 0,
                                        s);
}

int launch_spmv_dot32(const Mat& A, const SpmvConfig& c, const float* p, float* q,
                      double* pq_part, PcgState* st, hipStream_t s) {
    return launch_rows<float, ROW_DOT>(A, A.v32, c, p, q, nullptr, nullptr, nullptr, pq_part, st, 0,
                                       s);
}

void launch_spmv64(const Mat& A, const SpmvConfig& c, const double* x, double* y,
                   hipStream_t s) {
    launch_rows<double, ROW_PLAIN>(A, A.v, c, x, y, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                   s);
}

void launch_spmv32(const Mat& A, const SpmvConfig& c, const float* x, float* y,
                   hipStream_t s) {
    launch_rows<float, ROW_PLAIN>(A, A.v32, c, x, y, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                  s);
}

void launch_residual64(const Mat& A, const SpmvConfig& c, const double* b, const double* x,
                       double* r, double* partials, PcgState* st, int outer_mode, hipStream_t s) {
    const int nb = launch_rows<double, ROW_RESID>(A, A.v, c, x, r, b, nullptr, nullptr, partials, st,
                                                  outer_mode, s);
    hipLaunchKernelGGL(k_finalize_rows<ROW_RESID>, dim3(1), dim3(WG), 0, s, partials, nb, st,
                       outer_mode);
}

int launch_update64(int n, double* x, double* r, const double* p, const double* q,
                    const double* dinv, const double* pq_part, int nb_pq, double* rz_part, int it,
                    PcgState* st, hipStream_t s) {
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_update<double>, dim3(nb), dim3(WG), 0, s, n, x, r, p, q, dinv, pq_part,
                       nb_pq, rz_part, it, st);
    return nb;
}

int launch_update32(int n, float* x, float* r, const float* p, const float* q,
                    const float* dinv, const double* pq_part, int nb_pq, double* rz_part, int it,
                    PcgState* st, hipStream_t s) {
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_update<float>, dim3(nb), dim3(WG), 0, s, n, x, r, p, q, dinv, pq_part,
                       nb_pq, rz_part, it, st);
    return nb;
}

void launch_pupdate64(int n, double* p, const double* r, const double* dinv,
                      const double* rz_part, int nb_rz, int it, PcgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pupdate<double>, dim3(vec_blocks(n)), dim3(WG), 0, s, n, p, r, dinv,
                       rz_part, nb_rz, it, st);
}

void launch_pupdate32(int n, float* p, const float* r, const float* dinv, const double* rz_part,
                      int nb_rz, int it, PcgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pupdate<float>, dim3(vec_blocks(n)), dim3(WG), 0, s, n, p, r, dinv,
                       rz_part, nb_rz, it, st);
}

void launch_inner_start(int n, const double* r64, const PcgState* outer, float* r32, float* d32,
                        float* p32, const float* dinv32, double inner_tol, int maxit,
                        double* partials, PcgState* inner, hipStream_t s) {
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_inner_start, dim3(nb), dim3(WG), 0, s, n, r64, outer, r32, d32, p32,
                       dinv32, partials);
    hipLaunchKernelGGL(k_finalize_inner, dim3(1), dim3(WG), 0, s, partials, nb, outer, inner_tol,
                       maxit, inner);
}

void launch_refine_update(int n, double* x, const float* d32, const PcgState* outer,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_refine_update, dim3(vec_blocks(n)), dim3(WG), 0, s, n, x, d32, outer);
}

void launch_fill(double* v, int64_t n, double value, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(WG), 0, s, v, n, value);
}

void launch_cast32(const double* v, float* v32, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_cast32, dim3(grid1(n)), dim3(WG), 0, s, v, v32, n);
}

void launch_coef(const double* perf, double c0, double* coef, int64_t E, hipStream_t s) {
    if (E > 0) hipLaunchKernelGGL(k_coef, dim3(grid1(E)), dim3(WG), 0, s, perf, c0, coef, E);
}

void launch_scatter_dirichlet(const int32_t* ids, const double* vals, int64_t nD, double* gnode,
                              hipStream_t s) {
    if (nD > 0)
        hipLaunchKernelGGL(k_scatter_dirichlet, dim3(grid1(nD)), dim3(WG), 0, s, ids, vals, nD,
                           gnode);
}

void launch_set_dirichlet(const int32_t* ids, const double* gnode, int64_t nD, double* x,
                          hipStream_t s) {
    if (nD > 0)
        hipLaunchKernelGGL(k_set_dirichlet, dim3(grid1(nD)), dim3(WG), 0, s, ids, gnode, nD, x);
}

void launch_assemble_colour(int npe, int affine, const int32_t* elems, int count,
                            const int32_t* conn, const double* xyz, const Layout& L,
                            const int32_t* e2s, const double* mass, const double* stiff,
                            double* vals, hipStream_t s) {
    if (count <= 0) return;
    const int grid = grid1((int64_t)count * npe);
    if (npe == 8 && affine)
        hipLaunchKernelGGL((k_assemble<8, true>), dim3(grid), dim3(WG), 0, s, elems, count, conn,
                           xyz, L, e2s, mass, stiff, vals);
    else if (npe == 8)
        hipLaunchKernelGGL((k_assemble<8, false>), dim3(grid), dim3(WG), 0, s, elems, count, conn,
                           xyz, L, e2s, mass, stiff, vals);
    else
        hipLaunchKernelGGL((k_assemble<4, false>), dim3(grid), dim3(WG), 0, s, elems, count, conn,
                           xyz, L, e2s, mass, stiff, vals);
}

void launch_slot_map(int64_t E, int npe, const int32_t* conn, const Layout& L, int32_t* e2s,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_slot_map, dim3(grid1(E * npe)), dim3(WG), 0, s, E, npe, conn, L, e2s);
}

void launch_lift(int n, const Layout& L, double* vals, float* vals32, const uint8_t* isD,
                 const double* gnode, double* lift, double* dinv, float* dinv32, int do_lift,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_lift, dim3(grid1(n)), dim3(WG), 0, s, n, L, vals, vals32, isD, gnode,
                       lift, dinv, dinv32, do_lift);
}

void launch_sigma(int npe, int64_t E, const int32_t* conn, const double* T, const double* sigma0,
                  double alpha, double T_ref, double* sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_sigma, dim3(grid1(E)), dim3(WG), 0, s, npe, E, conn, T, sigma0, alpha,
                       T_ref, sigma);
}

void launch_bioheat_rhs_colour(int npe, int affine, const int32_t* elems, int count,
                               const int32_t* conn, const double* xyz, const double* T,
                               const double* V, const double* sigma, const double* perf,
                               double rho_c_dt, double T_a, int with_joule, double* rhs,
                               hipStream_t s) {
    if (count <= 0) return;
    const int grid = grid1((int64_t)count * npe);
    if (npe == 8 && affine)
        hipLaunchKernelGGL((k_bioheat_rhs<8, true>), dim3(grid), dim3(WG), 0, s, elems, count, conn,
                           xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, rhs);
    else if (npe == 8)
        hipLaunchKernelGGL((k_bioheat_rhs<8, false>), dim3(grid), dim3(WG), 0, s, elems, count,
                           conn, xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, rhs);
    else
        hipLaunchKernelGGL((k_bioheat_rhs<4, false>), dim3(grid), dim3(WG), 0, s, elems, count,
                           conn, xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, rhs);
}

void launch_finish_rhs(int n, const double* rhs, const double* lift, const uint8_t* isD,
                       double* b, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_rhs, dim3(grid1(n)), dim3(WG), 0, s, n, rhs, lift, isD, b);
}

}  // namespace rafem
