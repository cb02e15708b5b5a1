// HIP kernels for gfx950: element-parallel, colour-by-colour FEM assembly into the
// matrix layouts of the solver, Dirichlet lifting, and the coupled step's right-hand
// sides.  Elements of one colour share no node, so the threads of one launch never add
// into the same row: no atomics are needed.  These kernels run a few times per time
// step; the per-iteration solver kernels are in pcg.hip.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fem_device.hpp"
#include "internal.hpp"

namespace rafem {
namespace {

using namespace dev;


// ---------------------------------------------------------------------------
// Assembly helpers
// ---------------------------------------------------------------------------
__global__ void k_fill(double* __restrict__ v, int64_t n, double value) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) v[i] = value;
}

__global__ void k_fill32(float* __restrict__ v, int64_t n, float value) {
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

// Entry indices of the row-wise assembly: for every incidence slot t holding (e, a) (row
// conn[e][a]), byte b of r2j[t] is the index within that row of the entry of column
// conn[e][b], taken from the element-to-value map e2s.  Empty slots (n2e < 0) get 0.
__global__ __launch_bounds__(WG) void k_row_slots(int64_t total, int npe,
                                                  const int* __restrict__ n2e,
                                                  const int* __restrict__ conn,
                                                  const int* __restrict__ e2s,
                                                  const int* __restrict__ sptr,
                                                  uint64_t* __restrict__ r2j) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= total) return;
    const int ea = n2e[t];
    uint64_t p = 0;
    if (ea >= 0) {
        const int r = conn[ea];
        const int base = sptr[r / WAVE] + r % WAVE;
        for (int b = 0; b < npe; ++b)
            p |= (uint64_t)((e2s[(int64_t)ea * npe + b] - base) / WAVE) << (8 * b);
    }
    r2j[t] = p;
}

// Geometric constants of every element, fixed for the mesh's life: for a parallelepiped
// hex its metric C = detJ J^-1 J^-T and detJ, scaled as hex_row_scaled takes them
// (C00/72 C11/72 C22/72 C01/24 C02/24 C12/24 detJ/216); for a tet the gradients of its
// barycentric coordinates (4 x 3) and its volume.
template <int NPE>
__global__ __launch_bounds__(WG) void k_elem_geo(int64_t E, const int* __restrict__ conn,
                                                 const double* __restrict__ xyz,
                                                 double* __restrict__ geo) {
    const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (e >= E) return;
    double X[NPE][3];
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        const int node = conn[e * NPE + b];
#pragma unroll
        for (int d = 0; d < 3; ++d) X[b][d] = xyz[(int64_t)node * 3 + d];
    }
    if constexpr (NPE == 8) {
        double C[3][3];
        const double det = hex_affine_metric(X, C);
        double* g = geo + e * kGeoHex;
        g[0] = C[0][0] / 72.0;
        g[1] = C[1][1] / 72.0;
        g[2] = C[2][2] / 72.0;
        g[3] = C[0][1] / 24.0;
        g[4] = C[0][2] / 24.0;
        g[5] = C[1][2] / 24.0;
        g[6] = det / 216.0;
        g[7] = 0.0;
    } else {
        double G[4][3];
        const double V = tet_geometry(X, G);
        double* g = geo + e * kGeoTet;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[b * 3 + d] = G[b][d];
        g[12] = V;
        g[13] = g[14] = g[15] = 0.0;
    }
}

// Registers of one incidence's geometric constants: 8 doubles for a parallelepiped hex,
// 13 (of 16) for a tet; none for a general hex (its rows come from the node coordinates).
template <int NPE, bool AFFINE>
struct IncGeo {
    static constexpr int W = NPE == 4 ? 7 : (AFFINE ? 4 : 1);
    double2 v[W];
    double m, c;
};

template <int NPE, bool AFFINE>
__device__ __forceinline__ void load_inc(const RowAsm& a, int ea, IncGeo<NPE, AFFINE>& g) {
    const int e = ea / NPE;
    if constexpr (NPE == 4 || AFFINE) {
        const double2* src = reinterpret_cast<const double2*>(
            a.geo + (int64_t)e * (NPE == 4 ? kGeoTet : kGeoHex));
#pragma unroll
        for (int q = 0; q < IncGeo<NPE, AFFINE>::W; ++q) g.v[q] = src[q];
    }
    g.m = a.mass ? a.mass[e] : 0.0;
    g.c = a.stiff ? a.stiff[e] : 0.0;
}

// Row a of m M_e + c K_e of the incidence ea = e NPE + a.
template <int NPE, bool AFFINE>
__device__ __forceinline__ void inc_row(const RowAsm& a, int ea, const IncGeo<NPE, AFFINE>& g,
                                        double (&R)[NPE]) {
    const int ia = ea % NPE;
    if constexpr (NPE == 8 && AFFINE) {
        const double Cs[6] = {g.c * g.v[0].x, g.c * g.v[0].y, g.c * g.v[1].x,
                              g.c * g.v[1].y, g.c * g.v[2].x, g.c * g.v[2].y};
        hex_row_scaled(Cs, g.m * g.v[3].x, ia, R);
    } else if constexpr (NPE == 8) {
        const int e = ea / NPE;
        double X[8][3];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int node = a.conn[(int64_t)e * 8 + b];
#pragma unroll
            for (int d = 0; d < 3; ++d) X[b][d] = a.xyz[(int64_t)node * 3 + d];
        }
        double Kr[8], Mr[8];
        hex_rows(X, ia, Kr, Mr);
#pragma unroll
        for (int b = 0; b < 8; ++b) R[b] = g.m * Mr[b] + g.c * Kr[b];
    } else {
        double G[4][3];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            G[(2 * q) / 3][(2 * q) % 3] = g.v[q].x;
            G[(2 * q + 1) / 3][(2 * q + 1) % 3] = g.v[q].y;
        }
        const double V = g.v[6].x;
        double ga[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            ga[d] = ia == 0 ? G[0][d] : ia == 1 ? G[1][d] : ia == 2 ? G[2][d] : G[3][d];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double K = V * (ga[0] * G[b][0] + ga[1] * G[b][1] + ga[2] * G[b][2]);
            const double M = (ia == b ? 2.0 : 1.0) * V / 20.0;
            R[b] = g.m * M + g.c * K;
        }
    }
}

// Row-wise assembly: one wavefront per slab, lane l its row.  The slab's incidences are
// stored lane-interleaved (slot isptr[slab] + k WAVE + lane holds the k-th (e, a) of the
// lane's row, or -1), so their loads are coalesced; each lane adds the rows a M_e + c K_e
// of its incidences into the slab's values kept in LDS ([width][WAVE], sized at launch),
// loading the next incidence's constants while it computes the current one.  Then the
// row is lifted (as k_lift) and its values, their FP32 copy, the lift and the Jacobi
// inverse are written; every slot of the slab is written once, padding included (as 0).
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WAVE) void k_assemble_rows(RowAsm a) {
    extern __shared__ double acc[];
    const int lane = threadIdx.x;
    const int sl = xcd_block(blockIdx.x, gridDim.x);
    if (sl >= a.nslabs) return;
    const int base = a.sptr[sl];
    const int width = (a.sptr[sl + 1] - base) / WAVE;
    const int r = sl * WAVE + lane;
    for (int j = 0; j < width; ++j) acc[j * WAVE + lane] = 0.0;
    const int i0 = a.isptr[sl];
    const int kmax = (a.isptr[sl + 1] - i0) / WAVE;
    // incidence k (ea, jj, g) and the indices of incidence k + 1 (ea2, jj2)
    int ea = -1, ea2 = -1;
    uint64_t jj = 0, jj2 = 0;
    IncGeo<NPE, AFFINE> g;
    if (kmax > 0) {
        ea = a.n2e[i0 + lane];
        jj = a.r2j[i0 + lane];
        if (ea >= 0) load_inc(a, ea, g);
    }
    if (kmax > 1) {
        ea2 = a.n2e[i0 + WAVE + lane];
        jj2 = a.r2j[i0 + WAVE + lane];
    }
    for (int k = 0; k < kmax; ++k) {
        const int ea_n = ea2;
        const uint64_t jj_n = jj2;
        IncGeo<NPE, AFFINE> g_n;
        if (ea_n >= 0) load_inc(a, ea_n, g_n);
        ea2 = -1;
        if (k + 2 < kmax) {
            ea2 = a.n2e[i0 + (k + 2) * WAVE + lane];
            jj2 = a.r2j[i0 + (k + 2) * WAVE + lane];
        }
        if (ea >= 0) {
            double R[NPE];
            inc_row(a, ea, g, R);
#pragma unroll
            for (int b = 0; b < NPE; ++b) acc[((jj >> (8 * b)) & 0xff) * WAVE + lane] += R[b];
        }
        ea = ea_n;
        jj = jj_n;
        g = g_n;
    }
    // Lifting from the row's precomputed Dirichlet-column mask and diagonal entry index: the
    // column ids and the values g are read only for entries in Dirichlet columns.
    const bool drow = r < a.n && a.do_lift && a.isD[r];
    const uint64_t dm = (r < a.n && a.do_lift) ? a.dmask[r] : 0u;
    const int jd = r < a.n ? (int)a.jdiag[r] : 255;  // 255: none
    double diag = 0.0, acc_l = 0.0;
#pragma unroll 4
    for (int j = 0; j < width; ++j) {
        const int64_t pos = base + (int64_t)j * WAVE + lane;
        double v = acc[j * WAVE + lane];
        if (drow) {
            v = j == jd ? 1.0 : 0.0;
        } else if ((dm >> j) & 1u) {
            acc_l += v * a.gnode[a.scol[pos]];
            v = 0.0;
        }
        if (j == jd) diag = v;
        a.vals[pos] = v;
        if (a.vals32) a.vals32[pos] = (float)v;
    }
    if (r >= a.n) return;
    if (drow) diag = 1.0;
    if (a.do_lift && a.lift) a.lift[r] = drow ? a.gnode[r] : -acc_l;
    if (a.dinv) {
        const double inv = 1.0 / diag;
        a.dinv[r] = inv;
        if (a.dinv32) a.dinv32[r] = (float)inv;
    }
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
// Without a colour list (elems NULL) the threads cover elements 0 .. count-1 and store the
// term in rhs[e NPE + a] (per incidence) instead.
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
    const int e = elems ? elems[t / NPE] : t / NPE;
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
        // The 8 threads of an element (8 consecutive lanes) split the quadrature: thread a
        // evaluates the integrand at Gauss point a,
        //   s_a = detJ (sum_b N_b T~_b + sigma |grad V|^2),
        // and then forms rhs_a = sum_q N_a(q) s_q from the 8 values of its lane group.
        double xi, et, ze;
        gauss_point(a, xi, et, ze);
        double Ji[3][3];
        const double det = AFFINE ? hex_affine_jacobian(X, Ji) : hex_jacobian(X, xi, et, ze, Ji);
        double Nw = 0.0, gv0 = 0.0, gv1 = 0.0, gv2 = 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            double Nb, d0, d1, d2;
            hex_shape(b, xi, et, ze, Nb, d0, d1, d2);
            Nw += Nb * Tw[b];
            gv0 += Vb[b] * d0;
            gv1 += Vb[b] * d1;
            gv2 += Vb[b] * d2;
        }
        double gV[3];
        grad_x(Ji, gv0, gv1, gv2, gV);
        const double sq = det * (Nw + sg * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]));
        const int lane0 = (int)(threadIdx.x % WAVE) & ~7;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double s_q = __shfl(sq, lane0 + q, WAVE);
            double gx, gy, gz;
            gauss_point(q, gx, gy, gz);
            double Na, d0, d1, d2;
            hex_shape(a, gx, gy, gz, Na, d0, d1, d2);
            f += Na * s_q;
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
    if (elems) rhs[nodes[a]] += f;
    else rhs[t] = f;
}

// The same per-incidence terms for parallelepiped hexes from their stored constants (as
// k_elem_geo keeps them): with C = detJ J^-1 J^-T, detJ |grad V|^2 = grad_xi V^T C grad_xi V,
// so no Jacobian is inverted and no coordinates are read.  Thread (e, a) evaluates the
// integrand at Gauss point a and forms sum_q N_a(q) s_q from its lane group, as
// k_bioheat_rhs does.
__global__ __launch_bounds__(WG) void k_bioheat_rhs_geo(int count, const int* __restrict__ conn,
                                                        const double* __restrict__ geo,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ V,
                                                        const double* __restrict__ sigma,
                                                        const double* __restrict__ perf,
                                                        double rho_c_dt, double T_a,
                                                        int with_joule, double* __restrict__ rhs) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= count * 8) return;
    const int e = t / 8, a = t % 8;
    const double2* g = reinterpret_cast<const double2*>(geo + (int64_t)e * kGeoHex);
    const double2 g0 = g[0], g1 = g[1], g2 = g[2], g3 = g[3];
    const double src = perf[e] * T_a;
    const double sg = with_joule ? sigma[e] : 0.0;
    // each lane reads its own node (a coalesced read of conn); the group of 8 exchanges them
    const int lane0 = (int)(threadIdx.x % WAVE) & ~7;
    const int node_a = conn[(int64_t)e * 8 + a];
    const double Tw_a = rho_c_dt * T[node_a] + src;
    const double V_a = with_joule ? V[node_a] : 0.0;
    double xi, et, ze;
    gauss_point(a, xi, et, ze);
    double Nw = 0.0, gv0 = 0.0, gv1 = 0.0, gv2 = 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const double Tw = __shfl(Tw_a, lane0 + b, WAVE);
        const double Vb = __shfl(V_a, lane0 + b, WAVE);
        double Nb, d0, d1, d2;
        hex_shape(b, xi, et, ze, Nb, d0, d1, d2);
        Nw += Nb * Tw;
        gv0 += Vb * d0;
        gv1 += Vb * d1;
        gv2 += Vb * d2;
    }
    const double C00 = 72.0 * g0.x, C11 = 72.0 * g0.y, C22 = 72.0 * g1.x;
    const double C01 = 24.0 * g1.y, C02 = 24.0 * g2.x, C12 = 24.0 * g2.y, det = 216.0 * g3.x;
    const double quad = C00 * gv0 * gv0 + C11 * gv1 * gv1 + C22 * gv2 * gv2 +
                        2.0 * (C01 * gv0 * gv1 + C02 * gv0 * gv2 + C12 * gv1 * gv2);
    const double sq = det * Nw + sg * quad;
    double f = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double s_q = __shfl(sq, lane0 + q, WAVE);
        double gx, gy, gz;
        gauss_point(q, gx, gy, gz);
        double Na, d0, d1, d2;
        hex_shape(a, gx, gy, gz, Na, d0, d1, d2);
        f += Na * s_q;
    }
    rhs[t] = f;
}

// Right-hand side by rows from the per-incidence terms of k_bioheat_rhs: row r adds its
// node's incidences in the lane-interleaved order of the row-wise assembly (ascending
// element), then b = rhs + lift, or the lifted value on Dirichlet rows.
__global__ __launch_bounds__(WG) void k_rhs_rows(int n, const int* __restrict__ isptr,
                                                 const int* __restrict__ n2e,
                                                 const double* __restrict__ erhs,
                                                 const double* __restrict__ lift,
                                                 const uint8_t* __restrict__ isD,
                                                 double* __restrict__ b) {
    const int r = blockIdx.x * WG + threadIdx.x;
    if (r >= n) return;
    const int sl = r / WAVE, lane = r % WAVE;
    const int i0 = isptr[sl], kmax = (isptr[sl + 1] - i0) / WAVE;
    double sum = 0.0;
    for (int k0 = 0; k0 < kmax; k0 += 8) {  // eight incidences' loads in flight at once
        int ea[8];
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ea[u] = k0 + u < kmax ? n2e[i0 + (k0 + u) * WAVE + lane] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ea[u] >= 0 ? erhs[ea[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (ea[u] >= 0) sum += v[u];
    }
    b[r] = isD[r] ? lift[r] : sum + lift[r];
}

__global__ void k_finish_rhs(int n, const double* __restrict__ rhs,
                             const double* __restrict__ lift, const uint8_t* __restrict__ isD,
                             double* __restrict__ b) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < n) b[i] = isD[i] ? lift[i] : rhs[i] + lift[i];
}

inline int grid1(int64_t n) { return (int)((n + WG - 1) / WG); }

// Predictor: out = a + c (a - b), or a when b is NULL.
__global__ __launch_bounds__(WG) void k_extrapolate(int n, const double* __restrict__ a,
                                                    const double* __restrict__ b, double c,
                                                    double* __restrict__ out) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < n) out[i] = b ? a[i] + c * (a[i] - b[i]) : a[i];
}

// Polynomial predictor: out = sum_k w_k x_k over the `terms` (3 to 5) kept states, in order.
struct PolyArgs {
    const double* x[5];
    double w[5];
};

__global__ __launch_bounds__(WG) void k_extrapolate_poly(int n, int terms, PolyArgs a,
                                                         double* __restrict__ out) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    double v = a.w[0] * a.x[0][i] + a.w[1] * a.x[1][i] + a.w[2] * a.x[2][i];
    if (terms > 3) v += a.w[3] * a.x[3][i];
    if (terms > 4) v += a.w[4] * a.x[4][i];
    out[i] = v;
}

// Sums of (x - y)^2 and x^2: per-block partials, then one block adds them in order.
__global__ __launch_bounds__(WG) void k_change_norm_part(int n, const double* __restrict__ x,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ partials) {
    const int i = blockIdx.x * WG + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < n) {
        const double d = x[i] - y[i];
        v[0] = d * d;
        v[1] = x[i] * x[i];
    }
    store_partials<2>(v, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(WG) void k_change_norm_final(const double* __restrict__ partials,
                                                          int nb, double* __restrict__ norm2) {
    double tot[2];
    grid_totals<2>(partials, nb, tot);
    if (threadIdx.x == 0) {
        norm2[0] = tot[0];
        norm2[1] = tot[1];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_fill(double* v, int64_t n, double value, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(WG), 0, s, v, n, value);
}

void launch_fill32(float* v, int64_t n, float value, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill32, dim3(grid1(n)), dim3(WG), 0, s, v, n, value);
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

void launch_row_slots(int64_t total, int npe, const int32_t* n2e, const int32_t* conn,
                      const int32_t* e2s, const int32_t* sptr, uint64_t* r2j, hipStream_t s) {
    hipLaunchKernelGGL(k_row_slots, dim3(grid1(total)), dim3(WG), 0, s, total, npe, n2e, conn,
                       e2s, sptr, r2j);
}

void launch_elem_geo(int64_t E, int npe, const int32_t* conn, const double* xyz, double* geo,
                     hipStream_t s) {
    if (npe == 8) hipLaunchKernelGGL(k_elem_geo<8>, dim3(grid1(E)), dim3(WG), 0, s, E, conn, xyz, geo);
    else hipLaunchKernelGGL(k_elem_geo<4>, dim3(grid1(E)), dim3(WG), 0, s, E, conn, xyz, geo);
}

void launch_assemble_rows(int npe, int affine, const RowAsm& a, hipStream_t s) {
    const size_t lds = (size_t)a.width * WAVE * sizeof(double);
    const dim3 grid(a.nslabs), block(WAVE);
    if (npe == 8) {
        if (affine) hipLaunchKernelGGL((k_assemble_rows<8, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_assemble_rows<8, false>), grid, block, lds, s, a);
    } else {
        hipLaunchKernelGGL((k_assemble_rows<4, false>), grid, block, lds, s, a);
    }
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

void launch_bioheat_rhs_rows(int npe, int affine, int64_t E, const int32_t* conn,
                             const double* xyz, const double* geo, const double* T, const double* V,
                             const double* sigma, const double* perf, double rho_c_dt, double T_a,
                             int with_joule, double* erhs, int n, const int32_t* isptr,
                             const int32_t* n2e, const double* lift, const uint8_t* isD,
                             double* b, hipStream_t s) {
    const int grid = grid1(E * npe);
    const int cnt = (int)E;
    if (npe == 8 && affine && geo)
        hipLaunchKernelGGL(k_bioheat_rhs_geo, dim3(grid), dim3(WG), 0, s, cnt, conn, geo, T, V,
                           sigma, perf, rho_c_dt, T_a, with_joule, erhs);
    else if (npe == 8 && affine)
        hipLaunchKernelGGL((k_bioheat_rhs<8, true>), dim3(grid), dim3(WG), 0, s, nullptr, cnt,
                           conn, xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, erhs);
    else if (npe == 8)
        hipLaunchKernelGGL((k_bioheat_rhs<8, false>), dim3(grid), dim3(WG), 0, s, nullptr, cnt,
                           conn, xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, erhs);
    else
        hipLaunchKernelGGL((k_bioheat_rhs<4, false>), dim3(grid), dim3(WG), 0, s, nullptr, cnt,
                           conn, xyz, T, V, sigma, perf, rho_c_dt, T_a, with_joule, erhs);
    hipLaunchKernelGGL(k_rhs_rows, dim3(grid1(n)), dim3(WG), 0, s, n, isptr, n2e, erhs, lift, isD,
                       b);
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

void launch_extrapolate(int n, const double* a, const double* b, double c, double* out,
                        hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_extrapolate, dim3(grid1(n)), dim3(WG), 0, s, n, a, b, c, out);
}

void launch_extrapolate_poly(int n, int terms, const double* const* x, const double* w,
                             double* out, hipStream_t s) {
    PolyArgs a;
    for (int k = 0; k < 5; ++k) {
        a.x[k] = k < terms ? x[k] : x[0];
        a.w[k] = k < terms ? w[k] : 0.0;
    }
    if (n > 0)
        hipLaunchKernelGGL(k_extrapolate_poly, dim3(grid1(n)), dim3(WG), 0, s, n, terms, a, out);
}

void launch_change_norm(int n, const double* x, const double* y, double* partials,
                        double* norm2, hipStream_t s) {
    const int nb = std::max(1, grid1(n));
    hipLaunchKernelGGL(k_change_norm_part, dim3(nb), dim3(WG), 0, s, n, x, y, partials);
    hipLaunchKernelGGL(k_change_norm_final, dim3(1), dim3(WG), 0, s, partials, nb, norm2);
}

void launch_finish_rhs(int n, const double* rhs, const double* lift, const uint8_t* isD,
                       double* b, hipStream_t s) {
    hipLaunchKernelGGL(k_finish_rhs, dim3(grid1(n)), dim3(WG), 0, s, n, rhs, lift, isD, b);
}

}  // namespace rafem
