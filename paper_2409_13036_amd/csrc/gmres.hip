// Kernels of the monolithic (T, V) corrector for gfx950: Newton's method on the implicit
// coupled step, whose Jacobian has a full 2x2 block (T and V of both nodes) wherever two
// nodes share an element, solved by restarted GMRES(m) with right block-Jacobi
// preconditioning.
//
// Storage.  The block matrix reuses the node graph's SELL slabs: slot k of the scalar
// layout holds the four values (TT, TV, VT, VV) of its node pair as one double4, so the
// column offsets (shared lists, int16 deltas or absolute columns) are those of the scalar
// matrices and a wavefront reads 2 KB of values per entry.  Vectors interleave the two
// unknowns of a node (double2: x = T, y = V).  The mixed variant runs the Arnoldi process
// on float4 / float2 copies (sums in double) and keeps the restarts' true residual and the
// update in FP64.
//
// GMRES.  Arnoldi with classical Gram-Schmidt applied twice (CGS2), which needs three
// passes over the basis per step -- dots, update with the second dots, and the corrected
// normalisation -- instead of one reduction per basis vector.  The norm of the twice
// orthogonalised vector is ||w'||^2 - ||h2||^2 (w' = w - V h1, h2 = V^T w'), the small
// second correction being orthogonal to the result.  Every reduction is deterministic:
// per-block partial sums in fixed slots, added in a fixed order by the next kernel.  The
// Hessenberg column, its Givens rotations and the residual estimate are updated on the
// device by one thread, so a whole restart cycle is enqueued without host round trips; the
// host reads the solver state once per cycle.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fem_device.hpp"
#include "internal.hpp"

namespace rafem {
namespace {

using namespace dev;

inline int grid1(int64_t n) { return (int)((n + WG - 1) / WG); }

// ---------------------------------------------------------------------------
// Jacobian and residual, one thread per (element of one colour, local row a).
// ---------------------------------------------------------------------------
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_jac_assemble(JacArgs a) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= a.count * NPE) return;
    const int e = a.elems[t / NPE];
    const int ia = t % NPE;
    int nodes[NPE];
    double X[NPE][3], Tb[NPE], Vb[NPE], Tnb[NPE];
    double Tsum = 0.0;
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        nodes[b] = a.conn[(int64_t)e * NPE + b];
#pragma unroll
        for (int i = 0; i < 3; ++i) X[b][i] = a.xyz[(int64_t)nodes[b] * 3 + i];
        Tb[b] = a.T[nodes[b]];
        Vb[b] = a.V[nodes[b]];
        Tnb[b] = a.Tn[nodes[b]];
        Tsum += Tb[b];
    }
    const int row = nodes[ia];
    if (a.isD[row]) return;  // Dirichlet rows: identity, residual 0
    const double sig = a.sigma0[e] * (1.0 + a.alpha * (Tsum / NPE - a.T_ref));
    const double c = a.sigma0[e] * a.alpha / NPE;  // d sigma_e / d T_b
    const double mc = a.rho_c_dt + a.perf[e], kc = a.k_e[e];
    double Kr[NPE], Mr[NPE], Jr[NPE];  // Jr[b] = int N_a grad N_b . grad V
    double q = 0.0;                    // int N_a |grad V|^2
    if constexpr (NPE == 8) {
        if constexpr (AFFINE) hex_rows_affine(X, ia, Kr, Mr);
        else hex_rows(X, ia, Kr, Mr);
#pragma unroll
        for (int b = 0; b < 8; ++b) Jr[b] = 0.0;
        for (int g = 0; g < 8; ++g) {
            double xi, et, ze;
            gauss_point(g, xi, et, ze);
            double Ji[3][3];
            const double det = hex_jacobian(X, xi, et, ze, Ji);
            double gN[8][3], gV[3] = {0.0, 0.0, 0.0}, Na = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                double Nb, d0, d1, d2;
                hex_shape(b, xi, et, ze, Nb, d0, d1, d2);
                grad_x(Ji, d0, d1, d2, gN[b]);
#pragma unroll
                for (int i = 0; i < 3; ++i) gV[i] += Vb[b] * gN[b][i];
                if (b == ia) Na = Nb;
            }
            const double wN = det * Na;
            q += wN * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]);
#pragma unroll
            for (int b = 0; b < 8; ++b)
                Jr[b] += wN * (gN[b][0] * gV[0] + gN[b][1] * gV[1] + gN[b][2] * gV[2]);
        }
    } else {
        double G[4][3];
        const double vol = tet_geometry(X, G);
        double gV[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 3; ++i) gV[i] += Vb[b] * G[b][i];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            Kr[b] = vol * (G[ia][0] * G[b][0] + G[ia][1] * G[b][1] + G[ia][2] * G[b][2]);
            Mr[b] = (ia == b ? 2.0 : 1.0) * vol / 20.0;
            Jr[b] = 0.25 * vol * (G[b][0] * gV[0] + G[b][1] * gV[1] + G[b][2] * gV[2]);
        }
        q = 0.25 * vol * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]);
    }
    double KV = 0.0, AT = 0.0, Mw = 0.0;
    const double src = a.perf[e] * a.T_a;
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        KV += Kr[b] * Vb[b];
        AT += (mc * Mr[b] + kc * Kr[b]) * Tb[b];
        Mw += Mr[b] * (a.rho_c_dt * Tnb[b] + src);
    }
    a.R[2 * (int64_t)row] += a.rsign * (AT - Mw - sig * q);
    a.R[2 * (int64_t)row + 1] += a.rsign * (sig * KV);
    int start = 0, len = 0, stride = 1;
    if (!a.e2s) row_span(a.L, row, start, len, stride);
    const int64_t ps = a.plane_stride;
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        if (a.isD[nodes[b]]) continue;  // Dirichlet columns stay 0
        const int k = a.e2s ? a.e2s[((int64_t)e * NPE + ia) * NPE + b]
                            : find_slot(a.L.cols, start, len, stride, nodes[b]);
        double* p = a.vals + (int64_t)k * a.slot_mul;
        p[0] += mc * Mr[b] + kc * Kr[b] - c * q;
        p[ps] += -2.0 * sig * Jr[b];
        p[2 * ps] += c * KV;
        p[3 * ps] += sig * Kr[b];
    }
}

// Identity diagonal block of every Dirichlet row (the rest of those rows stays 0).
__global__ void k_jac_dirichlet(const int* __restrict__ dir_ids, int64_t nD, const Layout L,
                                double* __restrict__ vals, int slot_mul, int64_t plane_stride) {
    const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (k >= nD) return;
    const int d = dir_ids[k];
    int start, len, stride;
    row_span(L, d, start, len, stride);
    double* p = vals + (int64_t)find_slot(L.cols, start, len, stride, d) * slot_mul;
    p[0] = 1.0;
    p[3 * plane_stride] = 1.0;
}

// Inverse of every node's 2x2 diagonal block (block-Jacobi preconditioner).
__global__ __launch_bounds__(WG) void k_block_inv(int n, const Layout L,
                                                  const double4* __restrict__ vals,
                                                  double4* __restrict__ binv) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    int start, len, stride;
    row_span(L, i, start, len, stride);
    const double4 d = vals[find_slot(L.cols, start, len, stride, i)];
    const double det = d.x * d.w - d.y * d.z;
    binv[i] = make_double4(d.w / det, -d.y / det, -d.z / det, d.x / det);
}

// Vector element types: the FP64 path keeps double2 (a node's T and V) and double4 (a
// 2x2 block); the mixed path's Arnoldi process keeps float2 / float4.  Arithmetic on basis
// values is done in double after loading.
__device__ __forceinline__ double2 ld2(const double2 v) { return v; }
__device__ __forceinline__ double2 ld2(const float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double4 ld4(const double4 v) { return v; }
// The value a store of v into an X2 element keeps (rounding to float for the FP32 basis).
template <typename X2>
__device__ __forceinline__ double2 kept(double2 v) {
    if constexpr (sizeof(X2) == sizeof(float2)) return make_double2((float)v.x, (float)v.y);
    else return v;
}
__device__ __forceinline__ double4 ld4(const float4 v) { return make_double4(v.x, v.y, v.z, v.w); }

__device__ __forceinline__ double2 bj_apply(const double4 B, const double2 v) {
    return make_double2(B.x * v.x + B.y * v.y, B.z * v.x + B.w * v.y);
}

__device__ __forceinline__ bool cycle_over(const GmState* st) { return st->cyc_done || st->solved; }

// ---------------------------------------------------------------------------
// Block SpMV y = A x on the SELL slabs (kBsellSlabs slabs per workgroup, two per
// wavefront), in the precision of the values (V4: double4 or float4; X2 the matching
// vector element).  Skipped when the solve is over, or (arnoldi) when the cycle is.
// ---------------------------------------------------------------------------
constexpr int kBlockUnroll = 6;
constexpr int kBsellSlabs = 2 * NWAVES;

template <typename V4, typename X2>
struct BsellT {
    int n, nslabs;
    const int32_t* sptr;
    const int32_t* scol;
    const int16_t* sdel;
    const int32_t* sofs;
    const int32_t* soff;
    const V4* vals;
    const X2* x;
    X2* y;
    const GmState* st;
    int arnoldi;
};

template <int MODE, typename V4, typename X2>  // MODE 0: shared offsets, 1: int16 deltas, 2: columns
__device__ __forceinline__ X2 bsell_row(const BsellT<V4, X2>& a, int base, int width, int so,
                                        int r, int lane) {
    using T = decltype(X2::x);
    T ax = T(0), ay = T(0);
    const int rc = min(r, a.n - 1);
    for (int j = 0; j < width; j += kBlockUnroll) {
        int c[kBlockUnroll];
        V4 v[kBlockUnroll];
#pragma unroll
        for (int u = 0; u < kBlockUnroll; ++u) {
            const bool in = j + u < width;
            const int k = base + (j + u) * WAVE + lane;
            if constexpr (MODE == 0) c[u] = in ? r + a.soff[so + j + u] : rc;
            else if constexpr (MODE == 1) c[u] = in ? rc + (int)a.sdel[k] : rc;
            else c[u] = in ? a.scol[k] : rc;
            if (in) v[u] = a.vals[k];
            else v[u].x = v[u].y = v[u].z = v[u].w = T(0);
        }
        X2 x[kBlockUnroll];
#pragma unroll
        for (int u = 0; u < kBlockUnroll; ++u) x[u] = a.x[c[u]];
#pragma unroll
        for (int u = 0; u < kBlockUnroll; ++u) {
            ax += v[u].x * x[u].x + v[u].y * x[u].y;
            ay += v[u].z * x[u].x + v[u].w * x[u].y;
        }
    }
    X2 out;
    out.x = ax;
    out.y = ay;
    return out;
}

template <typename V4, typename X2>
__global__ __launch_bounds__(WG) void k_bsell(BsellT<V4, X2> a) {
    if (a.st && (a.st->solved || (a.arnoldi && a.st->cyc_done))) return;
    const int nblk = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nblk);
    const int lane = threadIdx.x % WAVE;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int s1 = min((blk + 1) * kBsellSlabs, a.nslabs);
    for (int sl = blk * kBsellSlabs + w; sl < s1; sl += NWAVES) {
        const int base = a.sptr[sl];
        const int width = (a.sptr[sl + 1] - base) / WAVE;
        const int so = a.sofs[sl];
        const int r = sl * WAVE + lane;
        X2 y;
        if (so >= 0) y = bsell_row<0>(a, base, width, so, r, lane);
        else if (a.sdel && so == -1) y = bsell_row<1>(a, base, width, so, r, lane);
        else y = bsell_row<2>(a, base, width, so, r, lane);
        if (r < a.n) a.y[r] = y;
    }
}

// ---------------------------------------------------------------------------
// GMRES vector kernels: one node (two values) per thread, partial sums per workgroup.
// ---------------------------------------------------------------------------
constexpr int kChunk = 8;

template <typename X2>
struct GmV {
    int n;
    X2* V;
    int64_t ldv;
    double* part;
    GmState* st;
};

// Per-block sums of the k values in lds[.][wave] -> part[i * nb + blk].
__device__ __forceinline__ void store_rows(double (*lds)[NWAVES], int k, double* part, int nb,
                                           int blk) {
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += WG) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NWAVES; ++j) s += lds[t][j];
        part[(int64_t)t * nb + blk] = s;
    }
}

// Wavefront sum of v into lds[i][wave].
__device__ __forceinline__ void wave_to_lds(double (*lds)[NWAVES], int i, double v) {
    v = wave_sum(v);
    if (threadIdx.x % WAVE == 0) lds[i][threadIdx.x / WAVE] = v;
}

template <typename X2>
__device__ __forceinline__ double2 basis(const GmV<X2>& a, int i, int node) {
    return ld2(a.V[(int64_t)i * a.ldv + node]);
}

// part[i] = V_i . w (i < k); NPT nodes per thread (one wavefront sum per vector covers
// 64 NPT nodes).
template <typename X2, int NPT>
__global__ __launch_bounds__(WG) void k_gm_dots(GmV<X2> a, int k, const X2* __restrict__ w) {
    if (cycle_over(a.st)) return;
    __shared__ double lds[kGmMaxM + 2][NWAVES];
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i0 = blk * WG * NPT + threadIdx.x;
    double2 wv[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        wv[q] = i0 + q * WG < a.n ? ld2(w[i0 + q * WG]) : make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        double2 v[kChunk][NPT];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
#pragma unroll
            for (int q = 0; q < NPT; ++q)
                v[u][q] = (c0 + u < k && i0 + q * WG < a.n) ? basis(a, c0 + u, i0 + q * WG)
                                                            : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            if (c0 + u < k) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NPT; ++q) t += v[u][q].x * wv[q].x + v[u][q].y * wv[q].y;
                wave_to_lds(lds, c0 + u, t);
            }
        }
    }
    store_rows(lds, k, a.part, nb, blk);
}

// out[b] = sum of partial row b (one workgroup per row, fixed order).
__global__ __launch_bounds__(WG) void k_gm_sum(const double* __restrict__ part, int nb,
                                               double* __restrict__ out, const GmState* st) {
    if (cycle_over(st)) return;
    const double* p = part + (int64_t)blockIdx.x * nb;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nb; t += WG) v[0] += p[t];
    block_sum<1>(v);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// w <- w - sum_i h1[i] V_i;  part[i] = V_i . w (i < k), part[k] = w . w.  KC > 0 keeps the
// basis values of the thread's NPT nodes in registers between the two loops (k <= KC).
template <int KC, typename X2, int NPT>
__global__ __launch_bounds__(WG) void k_gm_orth(GmV<X2> a, int k, const double* __restrict__ h1,
                                                X2* __restrict__ w) {
    if (cycle_over(a.st)) return;
    __shared__ double lds[kGmMaxM + 2][NWAVES];
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i0 = blk * WG * NPT + threadIdx.x;
    bool in[NPT];
    double2 wv[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        in[q] = i0 + q * WG < a.n;
        wv[q] = in[q] ? ld2(w[i0 + q * WG]) : make_double2(0.0, 0.0);
    }
    if constexpr (KC > 0) {
        X2 v[KC][NPT];  // raw basis values (float2 for the FP32 basis)
#pragma unroll
        for (int u = 0; u < KC; ++u)
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                if (u < k && in[q]) v[u][q] = a.V[(int64_t)u * a.ldv + i0 + q * WG];
                else v[u][q].x = v[u][q].y = 0;
            }
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            if (u < k) {
                const double h = h1[u];
#pragma unroll
                for (int q = 0; q < NPT; ++q) {
                    const double2 b = ld2(v[u][q]);
                    wv[q].x -= h * b.x;
                    wv[q].y -= h * b.y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            wv[q] = kept<X2>(wv[q]);  // the dots below use the stored w'
            if (in[q]) st2(&w[i0 + q * WG], wv[q]);
        }
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            if (u < k) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NPT; ++q) {
                    const double2 b = ld2(v[u][q]);
                    t += b.x * wv[q].x + b.y * wv[q].y;
                }
                wave_to_lds(lds, u, t);
            }
        }
    } else {
        for (int c0 = 0; c0 < k; c0 += kChunk) {
            double2 v[kChunk][NPT];
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
#pragma unroll
                for (int q = 0; q < NPT; ++q)
                    v[u][q] = (c0 + u < k && in[q]) ? basis(a, c0 + u, i0 + q * WG)
                                                    : make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                if (c0 + u < k) {
                    const double h = h1[c0 + u];
#pragma unroll
                    for (int q = 0; q < NPT; ++q) {
                        wv[q].x -= h * v[u][q].x;
                        wv[q].y -= h * v[u][q].y;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            wv[q] = kept<X2>(wv[q]);
            if (in[q]) st2(&w[i0 + q * WG], wv[q]);
        }
        for (int c0 = 0; c0 < k; c0 += kChunk) {
            double2 v[kChunk][NPT];
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
#pragma unroll
                for (int q = 0; q < NPT; ++q)
                    v[u][q] = (c0 + u < k && in[q]) ? basis(a, c0 + u, i0 + q * WG)
                                                    : make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                if (c0 + u < k) {
                    double t = 0.0;
#pragma unroll
                    for (int q = 0; q < NPT; ++q) t += v[u][q].x * wv[q].x + v[u][q].y * wv[q].y;
                    wave_to_lds(lds, c0 + u, t);
                }
            }
        }
    }
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NPT; ++q) t += wv[q].x * wv[q].x + wv[q].y * wv[q].y;
    wave_to_lds(lds, k, t);
    store_rows(lds, k + 1, a.part, nb, blk);
}

// Norm of the twice-orthogonalised vector from ||w'||^2 (h2[k]) and h2[0..k).
__device__ __forceinline__ double next_norm(const double* __restrict__ h2, int k) {
    double s = 0.0;
    for (int u = 0; u < k; ++u) s += h2[u] * h2[u];
    const double d = h2[k] - s;
    return d > 0.0 ? sqrt(d) : 0.0;
}

// v_k = (w' - sum_i h2[i] V_i) / h_{k,k-1};  z = M^-1 v_k (M^-1 in the basis' precision).
template <typename X2, typename B4>
__global__ __launch_bounds__(WG) void k_gm_next(GmV<X2> a, int k, const double* __restrict__ h2,
                                                const X2* __restrict__ w,
                                                const B4* __restrict__ binv, X2* __restrict__ z) {
    if (cycle_over(a.st)) return;
    const double hn = next_norm(h2, k);
    if (hn == 0.0) return;  // exact breakdown: the cycle ends here
    const int nb = gridDim.x;
    const int i = xcd_block(blockIdx.x, nb) * WG + threadIdx.x;
    if (i >= a.n) return;
    double2 wv = ld2(w[i]);
    for (int i0 = 0; i0 < k; i0 += kChunk) {
        double2 v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
            v[u] = i0 + u < k ? basis(a, i0 + u, i) : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            if (i0 + u < k) {
                const double h = h2[i0 + u];
                wv.x -= h * v[u].x;
                wv.y -= h * v[u].y;
            }
        }
    }
    const double2 vk = kept<X2>(make_double2(wv.x / hn, wv.y / hn));
    st2(&a.V[(int64_t)k * a.ldv + i], vk);
    st2(&z[i], bj_apply(ld4(binv[i]), vk));
}

// Hessenberg column j = (h1 + h2, h_{j+1,j}), earlier rotations, a new rotation, the
// rotated right-hand side and the residual estimate; ends the cycle when the estimate
// meets the tolerance, at the last column, on breakdown or at the iteration limit.
__global__ __launch_bounds__(WAVE) void k_gm_givens(GmSmall sm, int j,
                                                    const double* __restrict__ h1,
                                                    const double* __restrict__ h2, GmState* st) {
    if (cycle_over(st)) return;
    // the column, its second-pass part and the earlier rotations, loaded by all lanes at once
    __shared__ double col[kGmMaxM + 2], sec[kGmMaxM + 2], cs[kGmMaxM], sn[kGmMaxM];
    for (int i = threadIdx.x; i <= j + 1; i += WAVE) {
        const double b = h2[i];  // h2[j + 1] is ||w'||^2
        sec[i] = b;
        if (i <= j) col[i] = h1[i] + b;
    }
    for (int i = threadIdx.x; i < j; i += WAVE) {
        cs[i] = sm.cs[i];
        sn[i] = sm.sn[i];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int ld = sm.ldh;
    double* Hj = sm.H + (int64_t)j * ld;
    const double hn = next_norm(sec, j + 1);  // the same sum, in the same order, as k_gm_next
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
    }
    const double den = hypot(col[j], col[j + 1]);
    st->iters += 1;
    if (!(den > 0.0) || !isfinite(den)) {
        st->status = RAFEM_E_BREAKDOWN;
        st->solved = 1;
        st->cyc_done = 1;
        return;
    }
    const double c = col[j] / den, sj = col[j + 1] / den;
    sm.cs[j] = c;
    sm.sn[j] = sj;
    for (int i = 0; i < j; ++i) Hj[i] = col[i];
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    const double gj = sm.g[j];
    sm.g[j + 1] = -sj * gj;
    sm.g[j] = c * gj;
    const double est = fabs(sj * gj);
    st->est = est;
    if (st->iters <= sm.hist_cap && sm.hist) sm.hist[st->iters - 1] = est / st->bnorm;
    if (est <= st->tol * st->bnorm || st->iters >= st->maxit || j + 1 == st->m || hn == 0.0) {
        st->cyc_done = 1;
        st->jdone = j + 1;
    }
}

// y = H(0:k, 0:k)^-1 g(0:k), k = the cycle's steps (back substitution).  Up to
// kStageY steps the triangle is first loaded into LDS by all threads.
constexpr int kStageY = 64;

__global__ __launch_bounds__(WG) void k_gm_solve_y(GmSmall sm, const GmState* st) {
    if (st->solved) return;
    const int k = st->jdone;
    if (k <= kStageY) {
        __shared__ double H[kStageY][kStageY + 1], g[kStageY], y[kStageY];
        for (int t = threadIdx.x; t < k * k; t += WG) {
            const int l = t / k, i = t % k;  // column l, row i
            if (i <= l) H[i][l] = sm.H[(int64_t)l * sm.ldh + i];
        }
        for (int t = threadIdx.x; t < k; t += WG) g[t] = sm.g[t];
        __syncthreads();
        if (threadIdx.x != 0) return;
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[i][l] * y[l];
            y[i] = s / H[i][i];
            sm.y[i] = y[i];
        }
        return;
    }
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = sm.g[i];
        for (int l = i + 1; l < k; ++l) s -= sm.H[(int64_t)l * sm.ldh + i] * sm.y[l];
        sm.y[i] = s / sm.H[(int64_t)i * sm.ldh + i];
    }
}

// delta += M^-1 (sum_{i<k} y_i V_i), k = the cycle's steps (FP64 update and M^-1).
template <typename X2>
__global__ __launch_bounds__(WG) void k_gm_xupdate(GmV<X2> a, const double* __restrict__ y,
                                                   const double4* __restrict__ binv,
                                                   double2* __restrict__ delta) {
    if (a.st->solved) return;
    const int k = a.st->jdone;
    const int nb = gridDim.x;
    const int i = xcd_block(blockIdx.x, nb) * WG + threadIdx.x;
    if (i >= a.n || k == 0) return;
    double2 u = make_double2(0.0, 0.0);
    for (int i0 = 0; i0 < k; i0 += kChunk) {
        double2 v[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            v[c] = i0 + c < k ? basis(a, i0 + c, i) : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (i0 + c < k) {
                const double yc = y[i0 + c];
                u.x += yc * v[c].x;
                u.y += yc * v[c].y;
            }
        }
    }
    const double2 d = bj_apply(binv[i], u);
    double2 x = delta[i];
    x.x += d.x;
    x.y += d.y;
    delta[i] = x;
}

// r = b - w (w NULL: r = b); part[blk] = r . r  (FP64)
__global__ __launch_bounds__(WG) void k_gm_resid(int n, double* __restrict__ part,
                                                 const GmState* st, const double2* __restrict__ b,
                                                 const double2* __restrict__ w,
                                                 double2* __restrict__ r) {
    if (st->solved) return;
    __shared__ double lds[1][NWAVES];
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i = blk * WG + threadIdx.x;
    double2 rv = make_double2(0.0, 0.0);
    if (i < n) {
        rv = b[i];
        if (w) {
            const double2 wv = w[i];
            rv.x -= wv.x;
            rv.y -= wv.y;
        }
        r[i] = rv;
    }
    wave_to_lds(lds, 0, rv.x * rv.x + rv.y * rv.y);
    store_rows(lds, 1, part, nb, blk);
}

// Restart decision from the true residual norm (first: it is also ||b||).
__global__ __launch_bounds__(WG) void k_gm_restart(const double* __restrict__ part, int nb,
                                                   GmSmall sm, GmState* st, int first) {
    if (st->solved) return;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < nb; t += WG) v[0] += part[t];
    block_sum<1>(v);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(v[0]);
    if (first) st->bnorm = beta;
    st->relres_true = st->bnorm > 0.0 ? beta / st->bnorm : 0.0;
    if (!isfinite(beta)) {
        st->status = RAFEM_E_BREAKDOWN;
        st->solved = 1;
    } else if (beta <= st->tol * st->bnorm) {
        st->status = RAFEM_OK;
        st->solved = 1;
    } else if (st->iters >= st->maxit) {
        st->status = RAFEM_E_NOCONV;
        st->solved = 1;
    } else {
        st->beta = beta;
        sm.g[0] = beta;
        st->cyc_done = 0;
        st->jdone = 0;
        st->cycles += 1;
    }
}

// v_0 = r / beta (stored in the basis' precision);  z = M^-1 v_0.
template <typename X2, typename B4>
__global__ __launch_bounds__(WG) void k_gm_v0(GmV<X2> a, const double2* __restrict__ r,
                                              const B4* __restrict__ binv, X2* __restrict__ z) {
    if (a.st->solved) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * WG + threadIdx.x;
    if (i >= a.n) return;
    const double beta = a.st->beta;
    const double2 rv = r[i];
    const double2 v = kept<X2>(make_double2(rv.x / beta, rv.y / beta));
    st2(&a.V[i], v);
    st2(&z[i], bj_apply(ld4(binv[i]), v));
}

__global__ void k_gm_init(GmState* st, double tol, int maxit, int m) {
    if (threadIdx.x != 0) return;
    GmState s{};
    s.tol = tol;
    s.maxit = maxit;
    s.m = m;
    s.status = RAFEM_E_NOCONV;
    *st = s;
}

// T += delta.x, V += delta.y; part[blk] = (delta_T . delta_T, T . T) for the change norm.
__global__ __launch_bounds__(WG) void k_newton_apply(int n, const double2* __restrict__ delta,
                                                     double* __restrict__ T,
                                                     double* __restrict__ V,
                                                     double* __restrict__ part) {
    __shared__ double lds[2][NWAVES];
    const int nb = gridDim.x;
    const int blk = xcd_block(blockIdx.x, nb);
    const int i = blk * WG + threadIdx.x;
    double dd = 0.0, tt = 0.0;
    if (i < n) {
        const double2 d = delta[i];
        const double t = T[i] + d.x;
        T[i] = t;
        V[i] += d.y;
        dd = d.x * d.x;
        tt = t * t;
    }
    wave_to_lds(lds, 0, dd);
    wave_to_lds(lds, 1, tt);
    store_rows(lds, 2, part, nb, blk);
}

__global__ __launch_bounds__(WG) void k_newton_norm(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
    double v[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < nb; t += WG) {
        v[0] += part[t];
        v[1] += part[nb + t];
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_jac_assemble_colour(int npe, int affine, const JacArgs& a, hipStream_t s) {
    if (a.count <= 0) return;
    const int blocks = (int)(((int64_t)a.count * npe + WG - 1) / WG);
    if (npe == 8) {
        if (affine) hipLaunchKernelGGL((k_jac_assemble<8, true>), dim3(blocks), dim3(WG), 0, s, a);
        else hipLaunchKernelGGL((k_jac_assemble<8, false>), dim3(blocks), dim3(WG), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_jac_assemble<4, false>), dim3(blocks), dim3(WG), 0, s, a);
    }
}

void launch_jac_dirichlet(const int32_t* dir_ids, int64_t nD, const Layout& L, double* vals,
                          int slot_mul, int64_t plane_stride, hipStream_t s) {
    if (nD <= 0) return;
    hipLaunchKernelGGL(k_jac_dirichlet, dim3(grid1(nD)), dim3(WG), 0, s, dir_ids, nD, L, vals,
                       slot_mul, plane_stride);
}

void launch_block_inv(int n, const Layout& L, const double* vals4, double* binv, hipStream_t s) {
    hipLaunchKernelGGL(k_block_inv, dim3(grid1(n)), dim3(WG), 0, s, n, L,
                       reinterpret_cast<const double4*>(vals4), reinterpret_cast<double4*>(binv));
}

template <typename V4, typename X2>
BsellT<V4, X2> bsell_args(const BsellArgs& a) {
    return BsellT<V4, X2>{a.n, a.nslabs, a.sptr, a.scol, a.sdel, a.sofs, a.soff,
                          static_cast<const V4*>(a.vals), static_cast<const X2*>(a.x),
                          static_cast<X2*>(a.y), a.st, a.arnoldi};
}

void launch_bsell(const BsellArgs& a, hipStream_t s) {
    const int blocks = (a.nslabs + kBsellSlabs - 1) / kBsellSlabs;
    if (a.fp32)
        hipLaunchKernelGGL((k_bsell<float4, float2>), dim3(blocks), dim3(WG), 0, s,
                           bsell_args<float4, float2>(a));
    else
        hipLaunchKernelGGL((k_bsell<double4, double2>), dim3(blocks), dim3(WG), 0, s,
                           bsell_args<double4, double2>(a));
}

int gm_blocks(int n) { return grid1(n); }

template <typename X2>
GmV<X2> gmv(const GmVec& a) {
    return GmV<X2>{a.n, static_cast<X2*>(a.V), a.ldv, a.part, a.st};
}

void launch_gm_init(GmState* st, double tol, int maxit, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, s, st, tol, maxit, m);
}

// One node per thread for both bases (two nodes per thread for the FP32 basis, halving the
// wavefront sums per byte, measured no faster at m = 20 and slower for longer bases).
int launch_gm_dots(const GmVec& a, int k, const void* w, hipStream_t s) {
    const int nb = grid1(a.n);
    if (a.fp32)
        hipLaunchKernelGGL((k_gm_dots<float2, 1>), dim3(nb), dim3(WG), 0, s, gmv<float2>(a), k,
                           static_cast<const float2*>(w));
    else
        hipLaunchKernelGGL((k_gm_dots<double2, 1>), dim3(nb), dim3(WG), 0, s, gmv<double2>(a), k,
                           static_cast<const double2*>(w));
    return nb;
}

void launch_gm_sum(const double* part, int nb, int rows, double* out, const GmState* st,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_gm_sum, dim3(rows), dim3(WG), 0, s, part, nb, out, st);
}

template <typename X2, int NPT>
int orth_kc(const GmVec& a, int k, const double* h1, void* w, hipStream_t s) {
    const int nb = grid1((a.n + NPT - 1) / NPT);
    const dim3 g(nb), b(WG);
    const GmV<X2> v = gmv<X2>(a);
    X2* w2 = static_cast<X2*>(w);
    // register caches up to 32 values per node and thread; longer bases are read twice
    constexpr int kMaxCache = NPT == 1 ? 32 : 16;
    if (k <= 8) hipLaunchKernelGGL((k_gm_orth<8, X2, NPT>), g, b, 0, s, v, k, h1, w2);
    else if (k <= 16) hipLaunchKernelGGL((k_gm_orth<16, X2, NPT>), g, b, 0, s, v, k, h1, w2);
    else if (k <= kMaxCache) hipLaunchKernelGGL((k_gm_orth<32, X2, NPT>), g, b, 0, s, v, k, h1, w2);
    else hipLaunchKernelGGL((k_gm_orth<0, X2, NPT>), g, b, 0, s, v, k, h1, w2);
    return nb;
}

int launch_gm_orth(const GmVec& a, int k, const double* h1, void* w, hipStream_t s) {
    if (a.fp32) return orth_kc<float2, 1>(a, k, h1, w, s);
    return orth_kc<double2, 1>(a, k, h1, w, s);
}

void launch_gm_next(const GmVec& a, int k, const double* h2, const void* w, const void* binv,
                    void* z, hipStream_t s) {
    const dim3 g(grid1(a.n)), b(WG);
    if (a.fp32)
        hipLaunchKernelGGL((k_gm_next<float2, float4>), g, b, 0, s, gmv<float2>(a), k, h2,
                           static_cast<const float2*>(w), static_cast<const float4*>(binv),
                           static_cast<float2*>(z));
    else
        hipLaunchKernelGGL((k_gm_next<double2, double4>), g, b, 0, s, gmv<double2>(a), k, h2,
                           static_cast<const double2*>(w), static_cast<const double4*>(binv),
                           static_cast<double2*>(z));
}

void launch_gm_givens(const GmSmall& sm, int j, const double* h1, const double* h2, GmState* st,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(WAVE), 0, s, sm, j, h1, h2, st);
}

void launch_gm_solve_y(const GmSmall& sm, const GmState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_solve_y, dim3(1), dim3(WG), 0, s, sm, st);
}

void launch_gm_xupdate(const GmVec& a, const double* y, const double* binv, double* delta,
                       hipStream_t s) {
    const dim3 g(grid1(a.n)), b(WG);
    const double4* B = reinterpret_cast<const double4*>(binv);
    double2* d = reinterpret_cast<double2*>(delta);
    if (a.fp32) hipLaunchKernelGGL(k_gm_xupdate<float2>, g, b, 0, s, gmv<float2>(a), y, B, d);
    else hipLaunchKernelGGL(k_gm_xupdate<double2>, g, b, 0, s, gmv<double2>(a), y, B, d);
}

void launch_gm_resid(const GmVec& a, const double* b, const double* w, double* r, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_resid, dim3(grid1(a.n)), dim3(WG), 0, s, a.n, a.part,
                       (const GmState*)a.st, reinterpret_cast<const double2*>(b),
                       reinterpret_cast<const double2*>(w), reinterpret_cast<double2*>(r));
}

void launch_gm_restart(const double* part, int nb, const GmSmall& sm, GmState* st, int first,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_gm_restart, dim3(1), dim3(WG), 0, s, part, nb, sm, st, first);
}

void launch_gm_v0(const GmVec& a, const double* r, const void* binv, void* z, hipStream_t s) {
    const dim3 g(grid1(a.n)), b(WG);
    const double2* r2 = reinterpret_cast<const double2*>(r);
    if (a.fp32)
        hipLaunchKernelGGL((k_gm_v0<float2, float4>), g, b, 0, s, gmv<float2>(a), r2,
                           static_cast<const float4*>(binv), static_cast<float2*>(z));
    else
        hipLaunchKernelGGL((k_gm_v0<double2, double4>), g, b, 0, s, gmv<double2>(a), r2,
                           static_cast<const double4*>(binv), static_cast<double2*>(z));
}

void launch_newton_apply(int n, const double* delta, double* T, double* V, double* part,
                         double* norm2, hipStream_t s) {
    const int nb = grid1(n);
    hipLaunchKernelGGL(k_newton_apply, dim3(nb), dim3(WG), 0, s, n,
                       reinterpret_cast<const double2*>(delta), T, V, part);
    hipLaunchKernelGGL(k_newton_norm, dim3(1), dim3(WG), 0, s, part, nb, norm2);
}

}  // namespace rafem
