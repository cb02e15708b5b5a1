// Adjoint (reverse-mode) kernels of one coupled time step, for gradients of a
// lesion-temperature loss with respect to per-element conductivity k_e and perfusion w_e.
//
// Step n maps T^{n-1} to (V^n, T^n).  Given the adjoint load lambda on T^n, the reverse
// step solves A_T mu = lambda and K_sigma nu = (dF/dV)^T mu (both symmetric, so both are
// ordinary PCG solves), and then needs only element-local contractions:
//   dL/dk_e += -mu_e^T K_e T^n_e,   dL/dw_e += -mu_e^T M_e (T^n_e - T_a)
//   sbar_e   = mu_e^T J_e(V^n) - nu_e^T K_e V^n_e        (J_e: Joule load at unit sigma)
//   lambda_{n-1} = (rho c/dt) M mu + sum_e sbar_e sigma0_e alpha / npe on e's nodes.
// Per-element outputs are reduced over the element's lanes (no scatter, no colouring);
// node outputs are scattered colour by colour like the assembly.
#include <hip/hip_runtime.h>

#include "fem_device.hpp"
#include "internal.hpp"

namespace rafem {
namespace {

using namespace dev;

template <int NPE>
__device__ __forceinline__ void load_element(const int* __restrict__ conn,
                                             const double* __restrict__ xyz, int e,
                                             int (&nodes)[NPE], double (&X)[NPE][3]) {
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        nodes[b] = conn[(int64_t)e * NPE + b];
#pragma unroll
        for (int i = 0; i < 3; ++i) X[b][i] = xyz[(int64_t)nodes[b] * 3 + i];
    }
}

// Rows a of K_e and M_e.
template <int NPE, bool AFFINE>
__device__ __forceinline__ void element_rows(const double (&X)[NPE][3], int a, double (&Kr)[NPE],
                                             double (&Mr)[NPE]) {
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
}

// Sum over the NPE consecutive lanes of one element (all of them active).
template <int NPE>
__device__ __forceinline__ double element_sum(double v) {
#pragma unroll
    for (int off = NPE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, NPE);
    return v;
}

// grad_k[e] -= mu_e^T K_e T_e ; grad_w[e] -= mu_e^T M_e (T_e - T_a).  All elements.
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_vjp_params(int64_t E, const int* __restrict__ conn,
                                                   const double* __restrict__ xyz,
                                                   const double* __restrict__ mu,
                                                   const double* __restrict__ Tn, double T_a,
                                                   double* __restrict__ grad_k,
                                                   double* __restrict__ grad_w) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= E * NPE) return;  // whole elements only: E * NPE is a multiple of NPE
    const int e = (int)(t / NPE), a = (int)(t % NPE);
    int nodes[NPE];
    double X[NPE][3];
    load_element<NPE>(conn, xyz, e, nodes, X);
    double Kr[NPE], Mr[NPE];
    element_rows<NPE, AFFINE>(X, a, Kr, Mr);
    double kt = 0.0, mt = 0.0;
#pragma unroll
    for (int b = 0; b < NPE; ++b) {
        const double tb = Tn[nodes[b]];
        kt += Kr[b] * tb;
        mt += Mr[b] * (tb - T_a);
    }
    const double m = mu[nodes[a]];
    const double gk = element_sum<NPE>(m * kt);
    const double gw = element_sum<NPE>(m * mt);
    if (a == 0) {
        grad_k[e] -= gk;
        grad_w[e] -= gw;
    }
}

// Joule-load transpose product, one thread per (element of this colour, local node b):
//   nubar[node b] += int 2 sigma_e (sum_a mu_a N_a) grad N_b . grad V
//   sbar1[e]       = sum_b mu_b int N_b |grad V|^2
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_vjp_joule(const int* __restrict__ elems, int count,
                                                  const int* __restrict__ conn,
                                                  const double* __restrict__ xyz,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ mu,
                                                  const double* __restrict__ sigma,
                                                  double* __restrict__ nubar,
                                                  double* __restrict__ sbar1) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= count * NPE) return;
    const int e = elems[t / NPE];
    const int b = t % NPE;
    int nodes[NPE];
    double X[NPE][3], Vb[NPE], mb[NPE];
    load_element<NPE>(conn, xyz, e, nodes, X);
#pragma unroll
    for (int c = 0; c < NPE; ++c) {
        Vb[c] = V[nodes[c]];
        mb[c] = mu[nodes[c]];
    }
    const double sg = sigma[e];
    double out = 0.0, jb = 0.0;
    if constexpr (NPE == 8) {
        double Ji[3][3];
        double det = 0.0;
        if constexpr (AFFINE) det = hex_affine_jacobian(X, Ji);
        for (int q = 0; q < 8; ++q) {
            double xi, et, ze;
            gauss_point(q, xi, et, ze);
            if constexpr (!AFFINE) det = hex_jacobian(X, xi, et, ze, Ji);
            double muq = 0.0, gv0 = 0.0, gv1 = 0.0, gv2 = 0.0, Nb = 0.0, db[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                double Nc, d0, d1, d2;
                hex_shape(c, xi, et, ze, Nc, d0, d1, d2);
                muq += mb[c] * Nc;
                gv0 += Vb[c] * d0;
                gv1 += Vb[c] * d1;
                gv2 += Vb[c] * d2;
                if (c == b) {
                    Nb = Nc;
                    db[0] = d0;
                    db[1] = d1;
                    db[2] = d2;
                }
            }
            double gV[3], gb[3];
            grad_x(Ji, gv0, gv1, gv2, gV);
            grad_x(Ji, db[0], db[1], db[2], gb);
            out += det * 2.0 * sg * muq * (gb[0] * gV[0] + gb[1] * gV[1] + gb[2] * gV[2]);
            jb += det * Nb * (gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2]);
        }
    } else {
        double G[4][3];
        const double vol = tet_geometry(X, G);
        double gV[3] = {0.0, 0.0, 0.0}, msum = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            msum += mb[c];
#pragma unroll
            for (int i = 0; i < 3; ++i) gV[i] += Vb[c] * G[c][i];
        }
        const double q = gV[0] * gV[0] + gV[1] * gV[1] + gV[2] * gV[2];
        out = 2.0 * sg * msum * vol / 4.0 * (G[b][0] * gV[0] + G[b][1] * gV[1] + G[b][2] * gV[2]);
        jb = q * vol / 4.0;
    }
    nubar[nodes[b]] += out;
    const double s1 = element_sum<NPE>(mb[b] * jb);
    if (b == 0) sbar1[e] = s1;
}

// dsig[e] = (sbar1[e] - nu_e^T K_e V_e) sigma0_e alpha / npe.  All elements.
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_vjp_sigma(int64_t E, const int* __restrict__ conn,
                                                  const double* __restrict__ xyz,
                                                  const double* __restrict__ nu,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ sbar1,
                                                  const double* __restrict__ sigma0,
                                                  double alpha, double* __restrict__ dsig) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= E * NPE) return;
    const int e = (int)(t / NPE), a = (int)(t % NPE);
    int nodes[NPE];
    double X[NPE][3];
    load_element<NPE>(conn, xyz, e, nodes, X);
    double Kr[NPE], Mr[NPE];
    element_rows<NPE, AFFINE>(X, a, Kr, Mr);
    double kv = 0.0;
#pragma unroll
    for (int b = 0; b < NPE; ++b) kv += Kr[b] * V[nodes[b]];
    const double s = element_sum<NPE>(nu[nodes[a]] * kv);
    if (a == 0) dsig[e] = (sbar1[e] - s) * sigma0[e] * alpha / NPE;
}

// lam[node a] += rho_c_dt (M_e mu_e)_a + dsig[e].  One thread per (element of this colour, a).
template <int NPE, bool AFFINE>
__global__ __launch_bounds__(WG) void k_vjp_lambda(const int* __restrict__ elems, int count,
                                                   const int* __restrict__ conn,
                                                   const double* __restrict__ xyz,
                                                   const double* __restrict__ mu,
                                                   const double* __restrict__ dsig,
                                                   double rho_c_dt, double* __restrict__ lam) {
    const int t = blockIdx.x * WG + threadIdx.x;
    if (t >= count * NPE) return;
    const int e = elems[t / NPE];
    const int a = t % NPE;
    int nodes[NPE];
    double X[NPE][3];
    load_element<NPE>(conn, xyz, e, nodes, X);
    double Kr[NPE], Mr[NPE];
    element_rows<NPE, AFFINE>(X, a, Kr, Mr);
    double mm = 0.0;
#pragma unroll
    for (int b = 0; b < NPE; ++b) mm += Mr[b] * mu[nodes[b]];
    lam[nodes[a]] += rho_c_dt * mm + (dsig ? dsig[e] : 0.0);
}

// Lesion loss: partial sums of scale (T_i - T*_i)^2 per block, and grad_i = 2 scale (T_i - T*_i).
__global__ __launch_bounds__(WG) void k_loss(int64_t n, const int* __restrict__ ids,
                                             const double* __restrict__ target,
                                             const double* __restrict__ T, double scale,
                                             double* __restrict__ grad, double* partials) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        const double d = T[ids[i]] - target[i];
        v[0] = scale * d * d;
        grad[ids[i]] = 2.0 * scale * d;
    }
    store_partials<1>(v, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(WG) void k_loss_finalize(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ loss) {
    double tot[1];
    grid_totals<1>(partials, nb, tot);
    if (threadIdx.x == 0) loss[0] = tot[0];
}

inline int grid1(int64_t n) { return (int)((n + WG - 1) / WG); }

}  // namespace

#define RAFEM_DISPATCH(npe, affine, KERNEL, grid, s, ...)                                         \
    do {                                                                                           \
        if ((npe) == 8 && (affine))                                                                \
            hipLaunchKernelGGL((KERNEL<8, true>), dim3(grid), dim3(WG), 0, s, __VA_ARGS__);         \
        else if ((npe) == 8)                                                                       \
            hipLaunchKernelGGL((KERNEL<8, false>), dim3(grid), dim3(WG), 0, s, __VA_ARGS__);        \
        else                                                                                       \
            hipLaunchKernelGGL((KERNEL<4, false>), dim3(grid), dim3(WG), 0, s, __VA_ARGS__);        \
    } while (0)

void launch_vjp_params(int npe, int affine, int64_t E, const int32_t* conn, const double* xyz,
                       const double* mu, const double* Tn, double T_a, double* grad_k,
                       double* grad_w, hipStream_t s) {
    RAFEM_DISPATCH(npe, affine, k_vjp_params, grid1(E * npe), s, E, conn, xyz, mu, Tn, T_a, grad_k,
                   grad_w);
}

void launch_vjp_joule_colour(int npe, int affine, const int32_t* elems, int count,
                             const int32_t* conn, const double* xyz, const double* V,
                             const double* mu, const double* sigma, double* nubar, double* sbar1,
                             hipStream_t s) {
    if (count <= 0) return;
    RAFEM_DISPATCH(npe, affine, k_vjp_joule, grid1((int64_t)count * npe), s, elems, count, conn,
                   xyz, V, mu, sigma, nubar, sbar1);
}

void launch_vjp_sigma(int npe, int affine, int64_t E, const int32_t* conn, const double* xyz,
                      const double* nu, const double* V, const double* sbar1,
                      const double* sigma0, double alpha, double* dsig, hipStream_t s) {
    RAFEM_DISPATCH(npe, affine, k_vjp_sigma, grid1(E * npe), s, E, conn, xyz, nu, V, sbar1, sigma0,
                   alpha, dsig);
}

void launch_vjp_lambda_colour(int npe, int affine, const int32_t* elems, int count,
                              const int32_t* conn, const double* xyz, const double* mu,
                              const double* dsig, double rho_c_dt, double* lam, hipStream_t s) {
    if (count <= 0) return;
    RAFEM_DISPATCH(npe, affine, k_vjp_lambda, grid1((int64_t)count * npe), s, elems, count, conn,
                   xyz, mu, dsig, rho_c_dt, lam);
}

void launch_loss(int64_t n, const int32_t* ids, const double* target, const double* T,
                 double scale, double* grad, double* partials, double* loss, hipStream_t s) {
    const int nb = grid1(n);
    if (nb > 0)
        hipLaunchKernelGGL(k_loss, dim3(nb), dim3(WG), 0, s, n, ids, target, T, scale, grad,
                           partials);
    hipLaunchKernelGGL(k_loss_finalize, dim3(1), dim3(WG), 0, s, partials, nb, loss);
}

}  // namespace rafem
