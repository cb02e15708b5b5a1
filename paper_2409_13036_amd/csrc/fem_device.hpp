// Device helpers shared by the HIP translation units: launch geometry, deterministic
// block reductions, and element geometry (trilinear hex, linear tet).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace rafem {
namespace dev {

constexpr int WG = 256;
constexpr int WAVE = 64;
constexpr int NWAVES = WG / WAVE;
constexpr int NXCD = 8;

// Workgroups are dispatched round-robin over the XCDs; give XCD x the x-th contiguous
// share of the logical block indices.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
    const int xcd = bid % NXCD, idx = bid / NXCD;
    const int q = nb / NXCD, r = nb % NXCD;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// A double moved between lanes by one DPP pattern (both 32-bit halves; lanes without a
// source read 0).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order, returned to every lane: pairs and quads by quad
// permutations, rows of 16 by row shifts of 4 and 8 (lane 15 of a row holds its sum), then
// the rows by the row broadcasts of lanes 15 and 31 (lane 63 ends with the total).  All
// register-to-register: no LDS round trips.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x114>(v);  // row_shr:4
    v += dpp_move<0x118>(v);  // row_shr:8
    v += dpp_move<0x142>(v);  // row_bcast:15
    v += dpp_move<0x143>(v);  // row_bcast:31
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), WAVE - 1);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), WAVE - 1);
    return __hiloint2double(hi, lo);
}

// Sum K values over the block in a fixed order; result in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
    __shared__ double lds[K][NWAVES];
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = wave_sum(v[k]);
        if (lane == 0) lds[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int j = 0; j < NWAVES; ++j) s += lds[k][j];
            v[k] = s;
        }
    }
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Store this block's K sums as partials (no synchronisation with other blocks).
template <int K>
__device__ __forceinline__ void store_partials(double (&v)[K], double* partials, int slot,
                                               int nb) {
    block_sum<K>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) partials[k * nb + slot] = v[k];
    }
}

// Totals of the K partial arrays written by the previous kernel, in a fixed order that
// does not depend on the calling block; the result is returned to every thread.
template <int K>
__device__ __forceinline__ void grid_totals(const double* __restrict__ partials, int nb,
                                            double (&tot)[K]) {
    __shared__ double bcast[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += WG) s += partials[k * nb + i];
        tot[k] = s;
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


// Entries of row r: positions start + j * stride, j < len (CSR: stride 1; SELL: 64).
__device__ __forceinline__ void row_span(const Layout& L, int r, int& start, int& len,
                                         int& stride) {
    if (L.sell) {
        start = L.sptr[r / WAVE] + (r % WAVE);
        len = L.rlen[r];
        stride = WAVE;
    } else {
        start = L.rp[r];
        len = L.rp[r + 1] - start;
        stride = 1;
    }
}

// Position of column `col` in a row's ascending column list.
__device__ __forceinline__ int find_slot(const int* __restrict__ cols, int start, int len,
                                         int stride, int col) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (cols[start + m * stride] < col) lo = m + 1;
        else hi = m;
    }
    return start + lo * stride;
}

// Reference-cube corner signs of hex local node a in the ABI order
// (0,0,0),(1,0,0),(1,1,0),(0,1,0),(0,0,1),(1,0,1),(1,1,1),(0,1,1).
__device__ __forceinline__ double hsx(int a) { return ((a + 1) & 2) ? 1.0 : -1.0; }
__device__ __forceinline__ double hsy(int a) { return (a & 2) ? 1.0 : -1.0; }
__device__ __forceinline__ double hsz(int a) { return (a & 4) ? 1.0 : -1.0; }

// Trilinear shape function b and its reference gradient at (xi, et, ze).
__device__ __forceinline__ void hex_shape(int b, double xi, double et, double ze, double& N,
                                          double& d0, double& d1, double& d2) {
    const double sx = hsx(b), sy = hsy(b), sz = hsz(b);
    const double f0 = 1.0 + sx * xi, f1 = 1.0 + sy * et, f2 = 1.0 + sz * ze;
    N = 0.125 * f0 * f1 * f2;
    d0 = 0.125 * sx * f1 * f2;
    d1 = 0.125 * sy * f0 * f2;
    d2 = 0.125 * sz * f0 * f1;
}

// J[i][d] = dx_i/dxi_d at a Gauss point; returns det and Jinv[d][i] = dxi_d/dx_i.
__device__ __forceinline__ double hex_jacobian(const double (&X)[8][3], double xi, double et,
                                               double ze, double (&Ji)[3][3]) {
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        double N, d0, d1, d2;
        hex_shape(b, xi, et, ze, N, d0, d1, d2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            J[i][0] += X[b][i] * d0;
            J[i][1] += X[b][i] * d1;
            J[i][2] += X[b][i] * d2;
        }
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    // inverse of J: (J^-1)[d][i]
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

__device__ __forceinline__ void grad_x(const double (&Ji)[3][3], double d0, double d1, double d2,
                                       double (&g)[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = Ji[0][i] * d0 + Ji[1][i] * d1 + Ji[2][i] * d2;
}

constexpr double kGauss = 0.57735026918962576451;  // 1/sqrt(3)

__device__ __forceinline__ void gauss_point(int q, double& xi, double& et, double& ze) {
    xi = (q & 1) ? kGauss : -kGauss;
    et = (q & 2) ? kGauss : -kGauss;
    ze = (q & 4) ? kGauss : -kGauss;
}

// Row a of the stiffness and mass of hex element with corner coordinates X.
__device__ inline void hex_rows(const double (&X)[8][3], int a, double (&Kr)[8], double (&Mr)[8]) {
#pragma unroll
    for (int b = 0; b < 8; ++b) Kr[b] = Mr[b] = 0.0;
    for (int q = 0; q < 8; ++q) {
        double xi, et, ze;
        gauss_point(q, xi, et, ze);
        double Ji[3][3];
        const double det = hex_jacobian(X, xi, et, ze, Ji);
        double Na, a0, a1, a2, ga[3];
        hex_shape(a, xi, et, ze, Na, a0, a1, a2);
        grad_x(Ji, a0, a1, a2, ga);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            double Nb, b0, b1, b2, gb[3];
            hex_shape(b, xi, et, ze, Nb, b0, b1, b2);
            grad_x(Ji, b0, b1, b2, gb);
            Kr[b] += det * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
            Mr[b] += det * Na * Nb;
        }
    }
}

// Parallelepiped (affine) hex: constant Jacobian J = [x1-x0, x3-x0, x4-x0] / 2.  With
// C = detJ J^-1 J^-T the stiffness is K_ab = sum_de C_de I_ab^de, where the reference
// integrals of products of trilinear shape-function derivatives factor per axis:
//   I_ab^dd = (s_ad s_bd / 64) 2 p_e p_f,   I_ab^de = (s_ad s_be / 64) 4 p_f  (d != e),
// p_k = 2 + (2/3) s_ak s_bk, s = corner signs; and M_ab = detJ p_0 p_1 p_2 / 64.  These
// are the exact integrals, which the 2x2x2 Gauss rule reproduces on affine elements.
__device__ __forceinline__ double hex_affine_jacobian(const double (&X)[8][3],
                                                      double (&Ji)[3][3]) {
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        J[i][0] = 0.5 * (X[1][i] - X[0][i]);
        J[i][1] = 0.5 * (X[3][i] - X[0][i]);
        J[i][2] = 0.5 * (X[4][i] - X[0][i]);
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

// C = detJ J^-1 J^-T of a parallelepiped hex; returns detJ.
__device__ __forceinline__ double hex_affine_metric(const double (&X)[8][3], double (&C)[3][3]) {
    double Ji[3][3];
    const double det = hex_affine_jacobian(X, Ji);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 3; ++e)
            C[d][e] = det * (Ji[d][0] * Ji[e][0] + Ji[d][1] * Ji[e][1] + Ji[d][2] * Ji[e][2]);
    return det;
}

// Row a of K_e and M_e of a parallelepiped hex from its metric C and detJ.
__device__ __forceinline__ void hex_rows_metric(const double (&C)[3][3], double det, int a,
                                                double (&Kr)[8], double (&Mr)[8]) {
    const double sa[3] = {hsx(a), hsy(a), hsz(a)};
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const double sb[3] = {hsx(b), hsy(b), hsz(b)};
        double pk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) pk[k] = 2.0 + (2.0 / 3.0) * sa[k] * sb[k];
        double k_ab = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                double I;
                if (d == e) {
                    I = sa[d] * sb[d] * (1.0 / 32.0) * pk[(d + 1) % 3] * pk[(d + 2) % 3];
                } else {
                    const int f = 3 - d - e;
                    I = sa[d] * sb[e] * (1.0 / 16.0) * pk[f];
                }
                k_ab += C[d][e] * I;
            }
        }
        Kr[b] = k_ab;
        Mr[b] = det * pk[0] * pk[1] * pk[2] * (1.0 / 64.0);
    }
}

// A signed power of two, 2^e (e within the normal range), built from its bit pattern.
__device__ __forceinline__ double signed_pow2(int neg, int e) {
    return __hiloint2double((int)(((unsigned)neg << 31) | ((unsigned)(1023 + e) << 20)), 0);
}

// Row a of c K_e + m M_e of a parallelepiped hex from its scaled metric Cs = c (C00/72,
// C11/72, C22/72, C01/24, C02/24, C12/24) and ms = m detJ/216.  With t_k = s_ak s_bk and
// q_k = 3 + t_k (so p_k = 2 q_k / 3), the integrals above become
//   K_ab = sum_d (C_dd/72) t_d q_e q_f + sum_{d<e} (C_de/24) (s_ad s_be + s_ae s_bd) q_f,
//   M_ab = (detJ/216) q_0 q_1 q_2,
// whose integer factors are 0 or signed powers of two: each entry costs seven FMAs.
__device__ __forceinline__ void hex_row_scaled(const double (&Cs)[6], double ms, int a,
                                               double (&R)[8]) {
    const int ab[3] = {((a + 1) >> 1) & 1, (a >> 1) & 1, (a >> 2) & 1};  // corner sign bits
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bb[3] = {((b + 1) >> 1) & 1, (b >> 1) & 1, (b >> 2) & 1};
        int t[3];  // t_k = +1
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k] = ab[k] == bb[k];
        double v = ms * signed_pow2(0, 3 + t[0] + t[1] + t[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            v += Cs[d] * signed_pow2(!t[d], 2 + t[(d + 1) % 3] + t[(d + 2) % 3]);
        constexpr int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int d = pd[q], e = pe[q], f = 3 - d - e;
            const bool nz = (ab[d] == bb[e]) == (ab[e] == bb[d]);
            v += Cs[3 + q] * (nz ? signed_pow2(ab[d] != bb[e], 2 + t[f]) : 0.0);
        }
        R[b] = v;
    }
}

__device__ inline void hex_rows_affine(const double (&X)[8][3], int a, double (&Kr)[8],
                                double (&Mr)[8]) {
    double C[3][3];
    const double det = hex_affine_metric(X, C);
    hex_rows_metric(C, det, a, Kr, Mr);
}

// Tet: volume and constant gradients of the barycentric coordinates.
__device__ __forceinline__ double tet_geometry(const double (&X)[4][3], double (&G)[4][3]) {
    double J[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) J[i][c] = X[c + 1][i] - X[0][i];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    // rows of J^-1 are the gradients of barycentric coordinates 1..3
    G[1][0] = c00 * id;
    G[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    G[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    G[2][0] = c01 * id;
    G[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    G[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    G[3][0] = c02 * id;
    G[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    G[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
    for (int i = 0; i < 3; ++i) G[0][i] = -(G[1][i] + G[2][i] + G[3][i]);
    return det / 6.0;
}

}  // namespace dev
}  // namespace rafem
