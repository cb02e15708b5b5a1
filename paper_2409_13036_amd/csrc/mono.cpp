// Host drivers of the monolithic (T, V) corrector: Jacobian assembly on the step layout,
// restarted GMRES(m) with one host synchronisation per restart cycle (every Arnoldi step,
// Givens rotation and the restart decision run on the device), and the workspace.
#include "mono.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace rafem {

namespace {

constexpr int kWG = 256;  // threads of the per-node GMRES kernels

JacArgs jac_args(rafem_mesh m, const rafem_phys* phys, const double* k_e, const double* perf,
                 const double* sigma0, const double* Tn, const double* T, const double* V) {
    JacArgs a;
    a.conn = m->conn;
    a.xyz = m->xyz;
    a.isD = m->isD;
    a.Tn = Tn;
    a.T = T;
    a.V = V;
    a.k_e = k_e;
    a.perf = perf;
    a.sigma0 = sigma0;
    a.rho_c_dt = phys->rho_c / phys->dt;
    a.T_a = phys->T_a;
    a.alpha = phys->alpha_sigma;
    a.T_ref = phys->T_ref;
    return a;
}

void jac_colours(rafem_mesh m, JacArgs a, hipStream_t s) {
    for (int c = 0; c < m->n_colours; ++c) {
        const int off = m->colour_off[c];
        a.elems = m->colour_elems + off;
        a.count = m->colour_off[c + 1] - off;
        launch_jac_assemble_colour(m->npe, m->affine, a, s);
    }
}

// The small arrays of one solve, carved from m->gm_small.
struct Small {
    GmSmall sm;
    double *h1, *h2;
};

Small small_arrays(rafem_mesh m, int mm, double* hist, int hist_cap) {
    Small o;
    double* p = m->gm_small;
    o.sm.H = p;
    o.sm.ldh = mm + 1;
    p += (size_t)(kGmMaxM + 1) * kGmMaxM;
    o.sm.cs = p;
    p += kGmMaxM;
    o.sm.sn = p;
    p += kGmMaxM;
    o.sm.g = p;
    p += kGmMaxM + 1;
    o.sm.y = p;
    p += kGmMaxM;
    o.h1 = p;
    p += kGmMaxM + 1;
    o.h2 = p;
    o.sm.hist = hist;
    o.sm.hist_cap = hist ? hist_cap : 0;
    return o;
}

constexpr size_t kSmallDoubles = (size_t)(kGmMaxM + 1) * kGmMaxM + 2 * kGmMaxM + (kGmMaxM + 1) +
                                 kGmMaxM + (kGmMaxM + 1) + (kGmMaxM + 2);

}  // namespace

GmresOpts resolve_gmres(const rafem_gmres_opts* o) {
    GmresOpts g;
    if (o) {
        if (o->m > 0) g.m = o->m;
        if (o->max_iters > 0) g.maxit = o->max_iters;
        if (o->tol > 0.0) g.tol = o->tol;
        if (o->precision != RAFEM_FP64 && o->precision != RAFEM_MIXED)
            throw Error{RAFEM_E_ARG, "GMRES precision must be RAFEM_FP64 or RAFEM_MIXED"};
        g.precision = o->precision;
    }
    if (g.m > kGmMaxM) throw Error{RAFEM_E_ARG, "GMRES restart length exceeds RAFEM_GMRES_MAX_M"};
    if (!std::isfinite(g.tol) || g.tol >= 1.0)
        throw Error{RAFEM_E_ARG, "GMRES tol must be in (0, 1)"};
    return g;
}

void mono_ensure(rafem_mesh m, int mvec, bool fp32) {
    const int nb = gm_blocks((int)m->n);
    const size_t npad = (size_t)nb * kWG;
    if (fp32 && !m->mono_vals32) {
        auto f = [&](size_t count) { return static_cast<float*>(mesh_alloc(m, count * sizeof(float))); };
        m->mono_vals32 = f(4 * (size_t)m->sell_nnz);
        m->mono_binv32 = f(4 * npad);
    }
    if (!m->mono_vals) {
        auto d = [&](size_t count) { return static_cast<double*>(mesh_alloc(m, count * sizeof(double))); };
        m->mono_vals = d(4 * (size_t)m->sell_nnz);
        m->mono_rhs = d(2 * npad);
        m->mono_binv = d(4 * npad);
        m->mono_delta = d(2 * npad);
        m->gm_w = d(2 * npad);
        m->gm_z = d(2 * npad);
        m->gm_r = d(2 * npad);
        m->gm_part = d((size_t)(kGmMaxM + 2) * nb);
        m->gm_small = d(kSmallDoubles);
        m->gm_st = static_cast<GmState*>(mesh_alloc(m, sizeof(GmState)));
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(GmState)) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{RAFEM_E_NOMEM, "pinned host allocation failed"};
        }
        m->gm_st_host = static_cast<GmState*>(h);
    }
    if (mvec > m->gm_cap) {
        if (m->gm_V) {
            RAFEM_HIP(hipDeviceSynchronize());
            RAFEM_HIP(hipFree(m->gm_V));
            m->gm_V = nullptr;
            m->gm_cap = 0;
        }
        void* p = nullptr;
        const size_t bytes = (size_t)(mvec + 1) * npad * 2 * sizeof(double);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{RAFEM_E_NOMEM, "hipMalloc of the GMRES basis (" + std::to_string(bytes) +
                                           " bytes) failed"};
        }
        m->gm_V = static_cast<double*>(p);
        m->gm_cap = mvec;
    }
}

void mono_assemble(rafem_mesh m, const rafem_phys* phys, const double* k_e, const double* perf,
                   const double* sigma0, const double* Tn, const double* T, const double* V,
                   hipStream_t s) {
    const Layout SL = mesh_sell_layout(m);
    launch_fill(m->mono_vals, 4 * m->sell_nnz, 0.0, s);
    launch_fill(m->mono_rhs, 2 * m->n, 0.0, s);
    JacArgs a = jac_args(m, phys, k_e, perf, sigma0, Tn, T, V);
    a.L = SL;
    a.e2s = m->e2s;
    a.vals = m->mono_vals;
    a.slot_mul = 4;
    a.plane_stride = 1;
    a.R = m->mono_rhs;
    a.rsign = -1.0;
    jac_colours(m, a, s);
    launch_jac_dirichlet(m->dir_ids, m->nD, SL, m->mono_vals, 4, 1, s);
    launch_block_inv((int)m->n, SL, m->mono_vals, m->mono_binv, s);
    if (m->mono_vals32) {  // FP32 copies for the mixed Arnoldi process
        launch_cast32(m->mono_vals, m->mono_vals32, 4 * m->sell_nnz, s);
        launch_cast32(m->mono_binv, m->mono_binv32, 4 * m->n, s);
    }
    RAFEM_HIP(hipGetLastError());
}

void mono_export(rafem_mesh m, const rafem_phys* phys, const double* k_e, const double* perf,
                 const double* sigma0, const double* Tn, const double* T, const double* V,
                 double* planes, double* R, hipStream_t s) {
    const Layout CL = mesh_csr_layout(m);
    launch_fill(planes, 4 * m->nnz, 0.0, s);
    launch_fill(R, 2 * m->n, 0.0, s);
    JacArgs a = jac_args(m, phys, k_e, perf, sigma0, Tn, T, V);
    a.L = CL;
    a.e2s = nullptr;
    a.vals = planes;
    a.slot_mul = 1;
    a.plane_stride = m->nnz;
    a.R = R;
    a.rsign = 1.0;
    jac_colours(m, a, s);
    launch_jac_dirichlet(m->dir_ids, m->nD, CL, planes, 1, m->nnz, s);
    RAFEM_HIP(hipGetLastError());
}

rafem_status gmres_solve(rafem_mesh m, const double* b, double* x, const GmresOpts& o,
                         double* hist, int hist_cap, rafem_gmres_info* info, hipStream_t s) {
    const int n = (int)m->n;
    const int nb = gm_blocks(n);
    const Small sa = small_arrays(m, o.m, hist, hist_cap);
    const bool fp32 = o.precision == RAFEM_MIXED;
    if (fp32 && !m->mono_vals32) throw Error{RAFEM_E_STATE, "no FP32 copy of the Jacobian"};
    // the basis (and w, z) in the Arnoldi precision; restarts and the update in FP64
    GmVec a{n, m->gm_V, (int64_t)nb * kWG, m->gm_part, m->gm_st, fp32 ? 1 : 0};
    const void* binv_k = fp32 ? (const void*)m->mono_binv32 : (const void*)m->mono_binv;
    BsellArgs A;  // Arnoldi SpMV: z -> w
    A.n = n;
    A.nslabs = m->nslabs;
    A.sptr = m->sptr;
    A.scol = m->scol;
    A.sdel = m->sdel;
    A.sofs = m->sofs;
    A.soff = m->soff;
    A.vals = fp32 ? (const void*)m->mono_vals32 : (const void*)m->mono_vals;
    A.x = m->gm_z;
    A.y = m->gm_w;
    A.st = m->gm_st;
    A.arnoldi = 1;
    A.fp32 = fp32 ? 1 : 0;
    BsellArgs Ar = A;  // restart SpMV (FP64): x -> w
    Ar.vals = m->mono_vals;
    Ar.x = x;
    Ar.arnoldi = 0;
    Ar.fp32 = 0;
    launch_gm_init(m->gm_st, o.tol, o.maxit, o.m, s);
    launch_fill(x, 2 * m->n, 0.0, s);
    launch_gm_resid(a, b, nullptr, m->gm_r, s);
    launch_gm_restart(m->gm_part, nb, sa.sm, m->gm_st, 1, s);
    launch_gm_v0(a, m->gm_r, binv_k, m->gm_z, s);
    // the device ends the solve (tolerance, iteration limit or breakdown) within
    // maxit / m + 1 cycles; the bound below only guards the host loop
    const int max_cycles = o.maxit / o.m + 3;
    for (int cyc = 0;; ++cyc) {
        for (int j = 0; j < o.m; ++j) {
            const int k = j + 1;
            launch_bsell(A, s);
            const int nb1 = launch_gm_dots(a, k, m->gm_w, s);
            launch_gm_sum(m->gm_part, nb1, k, sa.h1, m->gm_st, s);
            const int nb2 = launch_gm_orth(a, k, sa.h1, m->gm_w, s);
            launch_gm_sum(m->gm_part, nb2, k + 1, sa.h2, m->gm_st, s);
            if (k < o.m) launch_gm_next(a, k, sa.h2, m->gm_w, binv_k, m->gm_z, s);
            launch_gm_givens(sa.sm, j, sa.h1, sa.h2, m->gm_st, s);
        }
        launch_gm_solve_y(sa.sm, m->gm_st, s);
        launch_gm_xupdate(a, sa.sm.y, m->mono_binv, x, s);
        launch_bsell(Ar, s);
        launch_gm_resid(a, b, m->gm_w, m->gm_r, s);
        launch_gm_restart(m->gm_part, nb, sa.sm, m->gm_st, 0, s);
        launch_gm_v0(a, m->gm_r, binv_k, m->gm_z, s);
        RAFEM_HIP(hipGetLastError());
        RAFEM_HIP(hipMemcpyAsync(m->gm_st_host, m->gm_st, sizeof(GmState), hipMemcpyDeviceToHost, s));
        RAFEM_HIP(hipStreamSynchronize(s));
        if (m->gm_st_host->solved) break;
        if (cyc >= max_cycles) throw Error{RAFEM_E_HIP, "GMRES did not end within its cycle bound"};
    }
    const GmState& h = *m->gm_st_host;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = h.status;
        info->iters = h.iters;
        info->cycles = h.cycles;
        info->relres = h.bnorm > 0.0 ? h.est / h.bnorm : 0.0;
        info->relres_true = h.relres_true;
    }
    return (rafem_status)h.status;
}

}  // namespace rafem
