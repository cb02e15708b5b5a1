// C ABI of the rafem library: argument checking, mesh lifetime, and the
// orchestration of assembly, solves and coupled time steps.  Every entry point
// catches all exceptions and turns them into a status code plus a thread-local
// message; nothing is enqueued after a failed host-side check.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "mono.hpp"
#include "solver.hpp"

namespace rafem {

namespace {
thread_local std::string g_error;

template <typename F>
rafem_status guard(F&& f) {
    try {
        clear_error();
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return RAFEM_E_NOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return RAFEM_E_HIP;
    } catch (...) {
        set_error("unknown error");
        return RAFEM_E_HIP;
    }
}

void require(bool ok, const char* what) {
    if (!ok) throw Error{RAFEM_E_ARG, what};
}

template <typename T>
T* dalloc(rafem_mesh m, size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{RAFEM_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    m->allocations.push_back(p);
    return static_cast<T*>(p);
}

void profile_off(rafem_mesh m) {
    for (hipEvent_t e : m->prof_ev) (void)hipEventDestroy(e);
    m->prof_ev.clear();
    m->prof_on = false;
}

void regions_off(rafem_mesh m) {
    for (hipEvent_t e : m->reg_ev) (void)hipEventDestroy(e);
    m->reg_ev.clear();
    m->reg_kind.clear();
    m->reg_on = false;
}

void free_mesh(rafem_mesh m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    profile_off(m);
    regions_off(m);
    for (auto& g : m->graphs) (void)hipGraphExecDestroy(g.exec);
    m->graphs.clear();
    if (m->gstream) (void)hipStreamDestroy(m->gstream);
    for (void* p : m->allocations) (void)hipFree(p);
    if (m->gm_V) (void)hipFree(m->gm_V);
    if (m->st_host) (void)hipHostFree(m->st_host);
    if (m->dd_log_host) (void)hipHostFree(m->dd_log_host);
    if (m->gm_st_host) (void)hipHostFree(m->gm_st_host);
    delete m;
}

void check_device(rafem_mesh m) {
    require(m != nullptr, "mesh is NULL");
    int d = -1;
    RAFEM_HIP(hipGetDevice(&d));
    if (d != m->device) throw Error{RAFEM_E_ARG, "the current HIP device is not the mesh's device"};
}

// Region timing: mark() opens an interval of the given region at the current point of
// the stream; flush() closes the step, waits for its last event and adds up the intervals.
constexpr int kRegAssembly = 0, kRegSolve = 1, kRegCheck = 2;

void region_mark(rafem_mesh m, int kind, hipStream_t s) {
    if (!m->reg_on) return;
    const size_t i = m->reg_kind.size();
    if (i >= m->reg_ev.size()) {
        hipEvent_t e;
        RAFEM_HIP(hipEventCreate(&e));
        m->reg_ev.push_back(e);
    }
    RAFEM_HIP(hipEventRecord(m->reg_ev[i], s));
    m->reg_kind.push_back(kind);
}

// Start of a step: drop boundaries left by a step that ended in an error.
void region_begin(rafem_mesh m) { m->reg_kind.clear(); }

void region_flush(rafem_mesh m, hipStream_t s) {
    if (!m->reg_on || m->reg_kind.empty()) return;
    region_mark(m, -1, s);
    const size_t n = m->reg_kind.size();
    RAFEM_HIP(hipEventSynchronize(m->reg_ev[n - 1]));
    for (size_t i = 0; i + 1 < n; ++i) {
        if (m->reg_kind[i] < 0) continue;
        float ms = 0.0f;
        RAFEM_HIP(hipEventElapsedTime(&ms, m->reg_ev[i], m->reg_ev[i + 1]));
        m->reg_ms[m->reg_kind[i]] += ms;
    }
    m->reg_kind.clear();
    m->reg_steps += 1;
}

Layout csr_layout(rafem_mesh m) {
    Layout L;
    L.sell = 0;
    L.rp = m->rp;
    L.cols = m->ci;
    return L;
}

Layout sell_layout(rafem_mesh m) {
    Layout L;
    L.sell = 1;
    L.sptr = m->sptr;
    L.rlen = m->rlen;
    L.cols = m->scol;
    return L;
}

// The step path keeps its matrices in the SELL layout.
Mat step_matrix(rafem_mesh m, const double* v, const float* v32) {
    Mat A;
    A.n = (int32_t)m->n;
    A.sell = 1;
    A.nslabs = m->nslabs;
    A.sptr = m->sptr;
    A.scol = m->scol;
    A.sdel = m->sdel;
    A.wide = m->sdel && m->int32_slabs > 0 ? 1 : 0;
    A.sofs = m->sofs;
    A.soff = m->soff;
    A.v = v;
    A.v32 = v32;
    return A;
}

Mat csr_matrix(rafem_mesh m, const int32_t* rp, const int32_t* ci, const double* v,
               const float* v32) {
    Mat A;
    A.n = (int32_t)m->n;
    A.sell = 0;
    A.rp = rp;
    A.ci = ci;
    A.v = v;
    A.v32 = v32;
    return A;
}

void assemble_into(rafem_mesh m, const Layout& L, int64_t count, const double* mass,
                   const double* stiff, double* vals, hipStream_t s) {
    launch_fill(vals, count, 0.0, s);
    const int32_t* e2s = L.sell ? m->e2s : nullptr;
    for (int c = 0; c < m->n_colours; ++c) {
        const int off = m->colour_off[c], cnt = m->colour_off[c + 1] - off;
        launch_assemble_colour(m->npe, m->affine, m->colour_elems + off, cnt, m->conn, m->xyz, L,
                               e2s, mass, stiff, vals, s);
    }
}

// Arguments of the row-wise assembly of one step-path matrix on the SELL layout.
RowAsm row_asm(rafem_mesh m, const double* mass, const double* stiff, const double* gnode,
               double* vals, float* vals32, double* lift, double* dinv, float* dinv32) {
    RowAsm a;
    a.n = (int)m->n;
    a.nslabs = m->nslabs;
    a.sptr = m->sptr;
    a.scol = m->scol;
    a.width = m->max_w;
    a.isptr = m->isptr;
    a.n2e = m->n2e;
    a.r2j = m->r2j;
    a.dmask = m->dmask;
    a.jdiag = m->jdiag;
    a.conn = m->conn;
    a.xyz = m->xyz;
    a.geo = m->geo;
    a.mass = mass;
    a.stiff = stiff;
    a.isD = m->isD;
    a.gnode = gnode;
    a.do_lift = m->nD > 0;
    a.vals = vals;
    a.vals32 = vals32;
    a.lift = lift;
    a.dinv = dinv;
    a.dinv32 = dinv32;
    return a;
}

// Bioheat matrix sum_e (rho_c/dt + w_e) M_e + k_e K_e, lifted with the values in m->gT.
void assemble_bioheat(rafem_mesh m, const rafem_phys* phys, const double* k_e,
                      const double* perf_e, hipStream_t s) {
    const Layout SL = sell_layout(m);
    launch_coef(perf_e, phys->rho_c / phys->dt, m->coefT, m->E, s);
    if (m->row_asm) {
        launch_assemble_rows(m->npe, m->affine,
                             row_asm(m, m->coefT, k_e, m->gT, m->valsT, m->valsT32, m->liftT,
                                     m->dinvT, m->dinvT32),
                             s);
    } else {
        assemble_into(m, SL, m->sell_nnz, m->coefT, k_e, m->valsT, s);
        launch_lift((int)m->n, SL, m->valsT, m->valsT32, m->isD, m->gT, m->liftT, m->dinvT,
                    m->dinvT32, m->nD > 0, s);
    }
    m->bioheat_ready = true;
    m->bioheat_dt = phys->dt;
}

// Potential matrix K_sigma(T) with sigma from the element means of T, lifted with m->gV.
void assemble_potential(rafem_mesh m, const rafem_phys* phys, const double* sigma0_e,
                        const double* T, hipStream_t s) {
    const Layout SL = sell_layout(m);
    launch_sigma(m->npe, m->E, m->conn, T, sigma0_e, phys->alpha_sigma, phys->T_ref, m->sigma, s);
    if (m->row_asm) {
        launch_assemble_rows(m->npe, m->affine,
                             row_asm(m, nullptr, m->sigma, m->gV, m->valsV, m->valsV32, m->liftV,
                                     m->dinvV, m->dinvV32),
                             s);
    } else {
        assemble_into(m, SL, m->sell_nnz, nullptr, m->sigma, m->valsV, s);
        launch_lift((int)m->n, SL, m->valsV, m->valsV32, m->isD, m->gV, m->liftV, m->dinvV,
                    m->dinvV32, m->nD > 0, s);
    }
    m->potential_ready = true;
}

// The buffers of device-driven steps (allocated once, by the handle's creation for a
// batch or by the first rafem_mesh_set_device_driven that turns them on).
void dd_alloc(rafem_mesh m) {
    if (m->dd_log) return;
    const size_t n = 3 * (size_t)m->S * kDdSlots;
    m->dd_log = dalloc<PcgState>(m, n);
    m->dd_x0 = dalloc<double>(m, (size_t)m->n);
    if (hipHostMalloc((void**)&m->dd_log_host, n * sizeof(PcgState), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        m->dd_log_host = nullptr;
        throw Error{RAFEM_E_NOMEM, "pinned host allocation failed"};
    }
}

Samples step_samples(rafem_mesh m) {
    return Samples{m->S, m->row_off, m->row_tab, m->max_sample_rows};
}
Samples whole_mesh(rafem_mesh m) { return Samples{1, m->row_off_one, nullptr, (int)m->n}; }

// Iteration counts a device-driven solve of this kind budgets for: per (inner) solve the
// larger of its counts in the last two solves of the kind.
std::vector<int> dd_counts(rafem_mesh m, int kind, bool mixed) {
    std::vector<int> c = m->hints[kind][mixed ? 1 : 0];
    const std::vector<int>& p = m->hints_prev[kind][mixed ? 1 : 0];
    for (size_t j = 0; j < c.size() && j < p.size(); ++j) c[j] = std::max(c[j], p[j]);
    return c;
}

void solve_any(rafem_mesh m, const SolveOpts& o, const Mat& A, const Samples& smp,
               const double* dinv, const float* dinv32, const double* b, double* x,
               rafem_solve_info* info, hipStream_t s, int kind) {
    // kind: which solve of a step (its own chunk hints per precision), or -1 for none
    const bool mixed = o.precision == RAFEM_MIXED;
    std::vector<int>* hints = kind >= 0 ? &m->hints[kind][mixed ? 1 : 0] : nullptr;
    if (hints) {
        const int k2 = mixed ? 1 : 0;
        m->hints_prev[kind][k2] = *hints;
        m->hints_prev_q[kind][k2] = m->hints_q[kind][k2];
        m->hints_q[kind][k2] = m->step_q;
    }
    if (mixed)
        pcg_mixed(m, A, smp, dinv, dinv32, b, x, o, info, s, hints);
    else
        pcg64(m, A, smp, dinv, b, x, o, info, s, hints);
}

void record_samples(rafem_mesh m, bool potential, bool mixed, const PcgState* h = nullptr);

// One solve of a coupled step (rafem_step's potential or bioheat solve), device-driven when
// the handle asks for it and the previous solve of this kind left its counts: the starting
// point is saved, the whole solve enqueued (dd_enqueue) and one poll of its logs decides
// whether it did exactly what the host-driven solve does; if not, the starting point is
// restored and the solve runs host-driven.  Either way the result, the info and the
// per-sample records are the host-driven solve's.
void solve_step(rafem_mesh m, const SolveOpts& o, const Mat& A, const double* dinv,
                const float* dinv32, const double* b, double* x, rafem_solve_info* info,
                hipStream_t s, int kind) {
    const bool mixed = o.precision == RAFEM_MIXED;
    const bool potential = kind == kSolvePotential;
    const int k2 = mixed ? 1 : 0;
    std::vector<int>& hints = m->hints[kind][k2];
    m->dd_used = 0;
    // budgets only from the last two solves of the kind when they started as this one does
    // (at a trajectory's start the predictor's order still rises and the counts move)
    const bool alike = m->hints_q[kind][k2] == m->step_q && m->hints_prev_q[kind][k2] == m->step_q;
    if (m->dd_on && m->tuned && !m->reg_on && alike && dd_ready(m, o, &hints)) {
        const size_t bytes = (size_t)m->n * sizeof(double);
        RAFEM_HIP(hipMemcpyAsync(m->dd_x0, x, bytes, hipMemcpyDeviceToDevice, s));
        const DdRecord r = dd_enqueue(m, A, step_samples(m), dinv, dinv32, b, x, o,
                                      dd_counts(m, kind, mixed), s);
        const size_t n = 3 * (size_t)m->S;
        RAFEM_HIP(hipMemcpyAsync(m->dd_log_host, m->dd_log, m->dd_used * n * sizeof(PcgState),
                                 hipMemcpyDeviceToHost, s));
        RAFEM_HIP(hipStreamSynchronize(s));
        std::vector<int> h = hints;
        const PcgState* hs = nullptr;
        if (dd_finish(m, r, o, info, &h, &hs)) {
            record_samples(m, potential, mixed, hs);
            m->hints_prev[kind][k2] = hints;
            m->hints_prev_q[kind][k2] = m->hints_q[kind][k2];
            m->hints_q[kind][k2] = m->step_q;
            hints = h;
            m->dd_solves += 1;
            return;
        }
        m->dd_redone += 1;
        RAFEM_HIP(hipMemcpyAsync(x, m->dd_x0, bytes, hipMemcpyDeviceToDevice, s));
    }
    solve_any(m, o, A, step_samples(m), dinv, dinv32, b, x, info, s, kind);
    record_samples(m, potential, mixed);
}

// Per-sample results of the solve that just finished (its last poll is in st_host).
void record_samples(rafem_mesh m, bool potential, bool mixed, const PcgState* h) {
    const int S = m->S;
    if (!h) h = m->st_host;
    for (int q = 0; q < S; ++q) {
        // a mixed solve's sample that fell back to FP64 PCG ends with that solve's state
        const bool fell = mixed && m->mixed_fell[q];
        const PcgState& main = (mixed && !fell) ? h[S + q] : h[q];
        rafem_solve_info& o = potential ? m->sample_info[q].V : m->sample_info[q].T;
        o.status = main.status;
        o.iters = mixed ? m->mixed_iters[q] : main.iters;
        o.outer = mixed ? (fell ? -h[S + q].iters : main.iters) : 0;
        o.launched = 0;
        o.relres = main.bb > 0.0 ? std::sqrt(main.rr / main.bb) : std::sqrt(main.rr);
        if (mixed && !fell) {
            o.relres_true = o.relres;
        } else {
            const PcgState& c = h[2 * S + q];
            o.relres_true = c.bb > 0.0 ? std::sqrt(c.rr / c.bb) : std::sqrt(c.rr);
        }
    }
}

// Everything rafem_mesh_create needs, for one mesh or the union of a batch (S samples,
// sample q owning nodes [node_off[q], node_off[q+1])).
rafem_mesh build_mesh(int64_t n_nodes, int64_t n_elems, int32_t npe, const double* xyz_h,
                      const int32_t* conn_h, const int32_t* dir_ids_h, int64_t n_dir, int S_,
                      const std::vector<int64_t>& node_off, const std::vector<int64_t>& elem_off,
                      const std::vector<int64_t>& dir_off) {
        check_conn(n_nodes, n_elems, npe, conn_h);
        for (int64_t k = 0; k < n_dir; ++k) {
            if (dir_ids_h[k] < 0 || dir_ids_h[k] >= n_nodes)
                throw Error{RAFEM_E_ARG, "Dirichlet id outside [0, n_nodes)"};
            if (k > 0 && dir_ids_h[k] <= dir_ids_h[k - 1])
                throw Error{RAFEM_E_ARG, "Dirichlet ids must be strictly increasing"};
        }
        for (int64_t i = 0; i < 3 * n_nodes; ++i)
            if (!std::isfinite(xyz_h[i])) throw Error{RAFEM_E_MESH, "non-finite node coordinate"};
        const bool affine = check_geometry(n_elems, npe, conn_h, xyz_h);
        HostStructure S = build_structure(n_nodes, n_elems, npe, conn_h);
        HostSell SL = build_sell(S, n_nodes, node_off);
        std::vector<int32_t> colour(n_elems);
        const int ncol = colour_elements(n_nodes, n_elems, npe, conn_h, colour.data());

        rafem_mesh m = new rafem_mesh_s();
        try {
            RAFEM_HIP(hipGetDevice(&m->device));
            m->n = n_nodes;
            m->E = n_elems;
            m->npe = npe;
            m->nnz = (int64_t)S.col_idx.size();
            m->nslabs = (int32_t)SL.nslabs;
            m->sell_nnz = (int64_t)SL.scol.size();
            m->nD = n_dir;
            m->n_colours = ncol;
            m->affine = (npe == 8 && affine) ? 1 : 0;
            m->spmv = choose_spmv_config(m->n, m->nnz);
            m->spmv32 = m->spmv;
            // elements grouped by colour, ascending id within a colour
            m->colour_off.assign(ncol + 1, 0);
            for (int64_t e = 0; e < n_elems; ++e) m->colour_off[colour[e] + 1]++;
            for (int c = 0; c < ncol; ++c) m->colour_off[c + 1] += m->colour_off[c];
            std::vector<int32_t> order(n_elems);
            std::vector<int32_t> fill(m->colour_off.begin(), m->colour_off.end() - 1);
            for (int64_t e = 0; e < n_elems; ++e) order[fill[colour[e]]++] = (int32_t)e;
            std::vector<uint8_t> isD(n_nodes, 0);
            for (int64_t k = 0; k < n_dir; ++k) isD[dir_ids_h[k]] = 1;

            const size_t N = (size_t)n_nodes, E = (size_t)n_elems, NNZ = (size_t)m->nnz;
            const size_t SNNZ = (size_t)m->sell_nnz;
            m->rp = dalloc<int32_t>(m, N + 1);
            m->ci = dalloc<int32_t>(m, NNZ);
            m->sptr = dalloc<int32_t>(m, (size_t)m->nslabs + 1);
            m->scol = dalloc<int32_t>(m, SNNZ);
            m->rlen = dalloc<int32_t>(m, N);
            m->e2s = dalloc<int32_t>(m, E * (size_t)npe * npe);
            if (!SL.sdel.empty()) m->sdel = dalloc<int16_t>(m, SNNZ);
            m->sofs = dalloc<int32_t>(m, (size_t)m->nslabs);
            m->soff = dalloc<int32_t>(m, std::max<size_t>(1, SL.soff.size()));
            for (int32_t o : SL.sofs) {
                m->shared_slabs += o >= 0 ? 1 : 0;
                m->int32_slabs += (o == -2 || (o == -1 && SL.sdel.empty())) ? 1 : 0;
            }
            // column data one product reads: per slab its pointers, then the shared offset
            // list (one entry per slot of a row) or a per-slot column offset
            m->index_bytes = 8 * (int64_t)m->nslabs;
            for (int64_t b = 0; b < m->nslabs; ++b) {
                const int64_t slots = SL.sptr[b + 1] - SL.sptr[b];
                if (SL.sofs[b] >= 0) m->index_bytes += 4 * (slots / 64);
                else m->index_bytes += (SL.sofs[b] == -1 && !SL.sdel.empty() ? 2 : 4) * slots;
            }
            m->conn = dalloc<int32_t>(m, E * npe);
            m->xyz = dalloc<double>(m, 3 * N);
            m->colour_elems = dalloc<int32_t>(m, E);
            m->dir_ids = dalloc<int32_t>(m, (size_t)n_dir);
            m->isD = dalloc<uint8_t>(m, N);
            m->gV = dalloc<double>(m, N);
            m->gT = dalloc<double>(m, N);
            m->gtmp = dalloc<double>(m, N);
            m->sigma = dalloc<double>(m, E);
            m->adj_mu = dalloc<double>(m, N);
            m->adj_nu = dalloc<double>(m, N);
            m->adj_sbar = dalloc<double>(m, E);
            m->adj_dsig = dalloc<double>(m, E);
            m->coefT = dalloc<double>(m, E);
            m->valsV = dalloc<double>(m, SNNZ);
            m->valsT = dalloc<double>(m, SNNZ);
            m->valsV32 = dalloc<float>(m, SNNZ);
            m->valsT32 = dalloc<float>(m, SNNZ);
            m->liftV = dalloc<double>(m, N);
            m->liftT = dalloc<double>(m, N);
            m->dinvV = dalloc<double>(m, N);
            m->dinvT = dalloc<double>(m, N);
            m->dinvV32 = dalloc<float>(m, N);
            m->dinvT32 = dalloc<float>(m, N);
            m->rhs = dalloc<double>(m, N);
            m->pc_Tn = dalloc<double>(m, N);
            m->pc_Vn = dalloc<double>(m, N);
            m->pc_Tk = dalloc<double>(m, N);
            for (int k = 0; k < rafem_mesh_s::kXgSlots; ++k) {  // extrapolation histories
                m->xg_T[k] = dalloc<double>(m, N);
                m->xg_V[k] = dalloc<double>(m, N);
            }
            m->pc_norm = dalloc<double>(m, 2);
            m->bT = dalloc<double>(m, N);
            m->r = dalloc<double>(m, N);
            m->p = dalloc<double>(m, N);
            m->q = dalloc<double>(m, N);
            m->dinv = dalloc<double>(m, N);
            m->r64 = dalloc<double>(m, N);
            m->r32 = dalloc<float>(m, N);
            m->p32 = dalloc<float>(m, N);
            m->q32 = dalloc<float>(m, N);
            m->d32 = dalloc<float>(m, N);
            m->dinv32 = dalloc<float>(m, N);
            m->partials = dalloc<double>(m, 3 * (N / 64 + 64));
            m->part_pq = dalloc<double>(m, N / 64 + 64);
            m->part_rz = dalloc<double>(m, 2 * (N / 64 + 64));
            m->part_sum = dalloc<double>(m, 3 * (size_t)S_);
            for (int q = 0; q < S_; ++q)
                m->max_sample_rows = std::max<int>(m->max_sample_rows,
                                                   (int)(node_off[q + 1] - node_off[q]));
            m->st = dalloc<PcgState>(m, 3 * (size_t)S_);
            m->itb = dalloc<int32_t>(m, 2);
            m->row_off = dalloc<int32_t>(m, (size_t)S_ + 1);
            m->row_off_one = dalloc<int32_t>(m, 2);
            if (hipHostMalloc((void**)&m->st_host, 3 * (size_t)S_ * sizeof(PcgState),
                              hipHostMallocDefault) !=
                hipSuccess) {
                (void)hipGetLastError();
                m->st_host = nullptr;
                throw Error{RAFEM_E_NOMEM, "pinned host allocation failed"};
            }
            std::memset(m->st_host, 0, 3 * (size_t)S_ * sizeof(PcgState));
            RAFEM_HIP(hipMemcpy(m->rp, S.row_ptr.data(), (N + 1) * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->ci, S.col_idx.data(), NNZ * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->sptr, SL.sptr.data(), SL.sptr.size() * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->scol, SL.scol.data(), SNNZ * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->rlen, SL.rlen.data(), N * 4, hipMemcpyHostToDevice));
            if (m->sdel)
                RAFEM_HIP(hipMemcpy(m->sdel, SL.sdel.data(), SNNZ * 2, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->sofs, SL.sofs.data(), SL.sofs.size() * 4, hipMemcpyHostToDevice));
            if (!SL.soff.empty())
                RAFEM_HIP(hipMemcpy(m->soff, SL.soff.data(), SL.soff.size() * 4,
                                    hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->conn, conn_h, E * npe * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->xyz, xyz_h, 3 * N * 8, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->colour_elems, order.data(), E * 4, hipMemcpyHostToDevice));
            if (n_dir > 0)
                RAFEM_HIP(hipMemcpy(m->dir_ids, dir_ids_h, (size_t)n_dir * 4, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->isD, isD.data(), N, hipMemcpyHostToDevice));
            RAFEM_HIP(hipMemcpy(m->st, m->st_host, 3 * (size_t)S_ * sizeof(PcgState),
                                hipMemcpyHostToDevice));
            std::vector<int32_t> roff(S_ + 1);
            for (int q = 0; q <= S_; ++q) roff[q] = (int32_t)node_off[q];
            const int32_t one[2] = {0, (int32_t)n_nodes};
            RAFEM_HIP(hipMemcpy(m->row_off, roff.data(), roff.size() * 4, hipMemcpyHostToDevice));
            if (S_ > 1) {
                // the sample of every kRowAlign-row block (every sample offset is a multiple)
                const int64_t nb = (n_nodes + kRowAlign - 1) / kRowAlign;
                std::vector<int32_t> tab(nb);
                for (int q = 0; q < S_; ++q)
                    for (int64_t b = node_off[q] / kRowAlign; b < (node_off[q + 1] + kRowAlign - 1) / kRowAlign && b < nb; ++b)
                        tab[b] = q;
                m->row_tab = dalloc<int32_t>(m, nb);
                RAFEM_HIP(hipMemcpy(m->row_tab, tab.data(), nb * 4, hipMemcpyHostToDevice));
            }
            RAFEM_HIP(hipMemcpy(m->row_off_one, one, 8, hipMemcpyHostToDevice));
            m->S = S_;
            m->node_off = node_off;
            m->elem_off = elem_off;
            m->dir_off = dir_off;
            m->sample_info.assign(S_, rafem_step_info{});
            m->use_graphs = S_ > 1;
            // a small mesh's iterations are launch-bound: its step solves replay graphs too
            m->graphs_small = S_ == 1 && n_nodes <= kGraphSmallRows;
            if (S_ > 1) {  // ensembles solve device-driven by default
                dd_alloc(m);
                m->dd_on = true;
            }
            launch_slot_map(m->E, m->npe, m->conn, sell_layout(m), m->e2s, nullptr);
            int32_t max_w = 0;
            for (int64_t b = 0; b < SL.nslabs; ++b)
                max_w = std::max(max_w, (SL.sptr[b + 1] - SL.sptr[b]) / 64);
            m->max_w = max_w;
            std::vector<int32_t> nptr, nlist, isptr;
            if (max_w <= kRowAsmMaxW) {
                node_elements(n_nodes, n_elems, npe, conn_h, nptr, nlist);
                // lane-interleaved incidences, each slab as deep as its busiest row
                isptr.assign(SL.nslabs + 1, 0);
                int64_t slots = 0;
                for (int64_t b = 0; b < SL.nslabs; ++b) {
                    int32_t deep = 0;
                    for (int64_t r = b * 64; r < std::min<int64_t>(n_nodes, b * 64 + 64); ++r)
                        deep = std::max(deep, nptr[r + 1] - nptr[r]);
                    slots += (int64_t)deep * 64;
                    if (slots > INT32_MAX) break;
                    isptr[b + 1] = (int32_t)slots;
                }
                if (slots > INT32_MAX) max_w = kRowAsmMaxW + 1;  // colour-by-colour instead
            }
            if (max_w <= kRowAsmMaxW) {
                std::vector<int32_t> n2e_s(std::max<int32_t>(1, isptr[SL.nslabs]), -1);
                for (int64_t r = 0; r < n_nodes; ++r)
                    for (int32_t k = nptr[r]; k < nptr[r + 1]; ++k)
                        n2e_s[isptr[r / 64] + (k - nptr[r]) * 64 + r % 64] = nlist[k];
                const size_t NS = n2e_s.size();
                m->isptr = dalloc<int32_t>(m, isptr.size());
                m->n2e = dalloc<int32_t>(m, NS);
                m->r2j = dalloc<uint64_t>(m, NS);
                RAFEM_HIP(hipMemcpy(m->isptr, isptr.data(), isptr.size() * 4,
                                    hipMemcpyHostToDevice));
                RAFEM_HIP(hipMemcpy(m->n2e, n2e_s.data(), NS * 4, hipMemcpyHostToDevice));
                launch_row_slots((int64_t)NS, npe, m->n2e, m->conn, m->e2s, m->sptr, m->r2j,
                                 nullptr);
                std::vector<uint64_t> dmask(N, 0u);
                std::vector<uint8_t> jdiag(N, 255);  // 255: no diagonal entry
                for (int64_t r = 0; r < n_nodes; ++r) {
                    const int64_t b0 = SL.sptr[r / 64] + r % 64;
                    for (int j = 0; j < SL.rlen[r]; ++j) {
                        const int32_t c = SL.scol[b0 + (int64_t)j * 64];
                        if (isD[c]) dmask[r] |= uint64_t{1} << j;
                        if (c == r) jdiag[r] = (uint8_t)j;
                    }
                }
                m->dmask = dalloc<uint64_t>(m, N);
                m->jdiag = dalloc<uint8_t>(m, N);
                RAFEM_HIP(hipMemcpy(m->dmask, dmask.data(), N * 8, hipMemcpyHostToDevice));
                RAFEM_HIP(hipMemcpy(m->jdiag, jdiag.data(), N, hipMemcpyHostToDevice));
                if (npe == 4 || m->affine) {
                    m->geo = dalloc<double>(m, E * (npe == 8 ? kGeoHex : kGeoTet));
                    launch_elem_geo(m->E, npe, m->conn, m->xyz, m->geo, nullptr);
                }
                m->erhs = dalloc<double>(m, E * npe);
                m->row_asm = true;
            }
            // The slab padding of the FP32 values is read by the FP32 SpMV (column = own
            // row) but never written by assembly or lifting: it must hold zeros.  (The FP64
            // values are cleared in full before every assembly.)
            launch_fill32(m->valsV32, SNNZ, 0.0f, nullptr);
            launch_fill32(m->valsT32, SNNZ, 0.0f, nullptr);
            RAFEM_HIP(hipGetLastError());
            RAFEM_HIP(hipDeviceSynchronize());
        } catch (...) {
            free_mesh(m);
            throw;
        }
    return m;
}

}  // namespace

void* mesh_alloc(rafem_mesh m, size_t bytes) { return dalloc<char>(m, bytes); }
Layout mesh_sell_layout(rafem_mesh m) { return sell_layout(m); }
Layout mesh_csr_layout(rafem_mesh m) { return csr_layout(m); }

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

}  // namespace rafem

using namespace rafem;

extern "C" {

const char* rafem_last_error(void) { return g_error.c_str(); }

int32_t rafem_abi_version(void) { return RAFEM_ABI_VERSION; }

rafem_status rafem_csr_structure(int64_t n_nodes, int64_t n_elems, int32_t npe,
                                 const int32_t* conn_h, int64_t* nnz_out, int32_t* row_ptr_h,
                                 int32_t* col_idx_h) {
    return guard([&]() -> rafem_status {
        require(nnz_out != nullptr, "nnz_out is NULL");
        check_conn(n_nodes, n_elems, npe, conn_h);
        HostStructure S = build_structure(n_nodes, n_elems, npe, conn_h);
        *nnz_out = (int64_t)S.col_idx.size();
        if (row_ptr_h && col_idx_h) {
            std::memcpy(row_ptr_h, S.row_ptr.data(), S.row_ptr.size() * sizeof(int32_t));
            std::memcpy(col_idx_h, S.col_idx.data(), S.col_idx.size() * sizeof(int32_t));
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_colour_elements(int64_t n_nodes, int64_t n_elems, int32_t npe,
                                   const int32_t* conn_h, int32_t* colour_h,
                                   int32_t* n_colours_out) {
    return guard([&]() -> rafem_status {
        require(colour_h != nullptr && n_colours_out != nullptr, "output is NULL");
        check_conn(n_nodes, n_elems, npe, conn_h);
        *n_colours_out = colour_elements(n_nodes, n_elems, npe, conn_h, colour_h);
        return RAFEM_OK;
    });
}

rafem_status rafem_rcm_order(int64_t n_nodes, int64_t n_elems, int32_t npe,
                             const int32_t* conn_h, int32_t* order_h) {
    return guard([&]() -> rafem_status {
        require(order_h != nullptr, "order is NULL");
        check_conn(n_nodes, n_elems, npe, conn_h);
        const HostStructure S = build_structure(n_nodes, n_elems, npe, conn_h);
        const std::vector<int32_t> order = rcm_order(n_nodes, S);
        std::memcpy(order_h, order.data(), order.size() * sizeof(int32_t));
        return RAFEM_OK;
    });
}

rafem_status rafem_degree_sort(int64_t n_nodes, int64_t n_elems, int32_t npe,
                               const int32_t* conn_h, int64_t window, int32_t* order_h) {
    return guard([&]() -> rafem_status {
        require(order_h != nullptr, "order is NULL");
        require(window >= 1, "window must be >= 1");
        check_conn(n_nodes, n_elems, npe, conn_h);
        std::vector<char> seen(n_nodes, 0);
        for (int64_t k = 0; k < n_nodes; ++k) {
            require(order_h[k] >= 0 && order_h[k] < n_nodes && !seen[order_h[k]],
                    "order is not a permutation of the nodes");
            seen[order_h[k]] = 1;
        }
        const HostStructure S = build_structure(n_nodes, n_elems, npe, conn_h);
        degree_sort(n_nodes, S, window, order_h);
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_create(int64_t n_nodes, int64_t n_elems, int32_t npe, const double* xyz_h,
                               const int32_t* conn_h, const int32_t* dir_ids_h, int64_t n_dir,
                               rafem_mesh* out) {
    return guard([&]() -> rafem_status {
        require(out != nullptr, "out is NULL");
        require(xyz_h != nullptr, "xyz is NULL");
        require(n_dir >= 0 && n_dir <= n_nodes, "n_dir out of range");
        require(n_dir == 0 || dir_ids_h != nullptr, "dir_ids is NULL");
        *out = nullptr;
        *out = build_mesh(n_nodes, n_elems, npe, xyz_h, conn_h, dir_ids_h, n_dir, 1, {0, n_nodes},
                          {0, n_elems}, {0, n_dir});
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_create_batch(int32_t n_samples, const int64_t* n_nodes,
                                     const int64_t* n_elems, int32_t npe,
                                     const double* const* xyz_h, const int32_t* const* conn_h,
                                     const int32_t* const* dir_ids_h, const int64_t* n_dir,
                                     rafem_mesh* out) {
    return guard([&]() -> rafem_status {
        require(out != nullptr, "out is NULL");
        require(n_samples >= 1 && n_samples <= 4096, "n_samples out of range");
        require(n_nodes && n_elems && xyz_h && conn_h && n_dir, "NULL argument");
        require(npe == 8 || npe == 4, "nodes_per_elem must be 8 (hex) or 4 (tet)");
        *out = nullptr;
        const int S_ = n_samples;
        // sample q: its nodes, then padding up to a multiple of kRowAlign; padding nodes have
        // no element and are Dirichlet nodes (their rows lift to the identity)
        std::vector<int64_t> node_off(S_ + 1, 0), elem_off(S_ + 1, 0), dir_off(S_ + 1, 0);
        for (int q = 0; q < S_; ++q) {
            require(n_nodes[q] > 0 && n_elems[q] > 0 && n_dir[q] >= 0 && n_dir[q] <= n_nodes[q],
                    "sample size out of range");
            require(xyz_h[q] && conn_h[q] && (n_dir[q] == 0 || dir_ids_h[q]), "NULL sample array");
            const int64_t padded = (n_nodes[q] + kRowAlign - 1) / kRowAlign * kRowAlign;
            node_off[q + 1] = node_off[q] + padded;
            elem_off[q + 1] = elem_off[q] + n_elems[q];
            dir_off[q + 1] = dir_off[q] + n_dir[q] + (padded - n_nodes[q]);
        }
        require(node_off[S_] < INT32_MAX && elem_off[S_] * npe < INT32_MAX, "batch too large");
        const int64_t N = node_off[S_], E = elem_off[S_], ND = dir_off[S_];
        std::vector<double> xyz(3 * N, 0.0);
        std::vector<int32_t> conn(E * npe), dirs(ND);
        for (int q = 0; q < S_; ++q) {
            const int64_t no = node_off[q], nq = n_nodes[q];
            std::memcpy(xyz.data() + 3 * no, xyz_h[q], 3 * nq * sizeof(double));
            for (int64_t i = nq; i < node_off[q + 1] - no; ++i)
                for (int c = 0; c < 3; ++c) xyz[3 * (no + i) + c] = xyz_h[q][c];
            for (int64_t k = 0; k < n_elems[q] * npe; ++k) {
                const int32_t v = conn_h[q][k];
                if (v < 0 || v >= nq) throw Error{RAFEM_E_MESH, "sample element refers to a node out of range"};
                conn[elem_off[q] * npe + k] = (int32_t)(v + no);
            }
            int64_t d = dir_off[q];
            for (int64_t k = 0; k < n_dir[q]; ++k) {
                if (dir_ids_h[q][k] < 0 || dir_ids_h[q][k] >= nq ||
                    (k > 0 && dir_ids_h[q][k] <= dir_ids_h[q][k - 1]))
                    throw Error{RAFEM_E_ARG, "sample Dirichlet ids must be increasing and in range"};
                dirs[d++] = (int32_t)(dir_ids_h[q][k] + no);
            }
            for (int64_t i = no + nq; i < node_off[q + 1]; ++i) dirs[d++] = (int32_t)i;
        }
        *out = build_mesh(N, E, npe, xyz.data(), conn.data(), dirs.data(), ND, S_, node_off,
                          elem_off, dir_off);
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_sample_layout(rafem_mesh m, int64_t* node_off, int64_t* elem_off,
                                      int64_t* dir_off) {
    return guard([&]() -> rafem_status {
        require(m != nullptr, "mesh is NULL");
        for (int q = 0; q <= m->S; ++q) {
            if (node_off) node_off[q] = m->node_off[q];
            if (elem_off) elem_off[q] = m->elem_off[q];
            if (dir_off) dir_off[q] = m->dir_off[q];
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_sample_info(rafem_mesh m, int32_t sample, rafem_step_info* out) {
    return guard([&]() -> rafem_status {
        require(m != nullptr && out != nullptr, "NULL argument");
        require(sample >= 0 && sample < m->S, "sample out of range");
        *out = m->sample_info[sample];
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_set_graphs(rafem_mesh m, int32_t enable) {
    return guard([&]() -> rafem_status {
        check_device(m);
        m->use_graphs = enable != 0;
        m->graphs_small = false;  // an explicit choice replaces the size rule
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_set_device_driven(rafem_mesh m, int32_t enable, double budget_scale) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(budget_scale == 0.0 || (budget_scale > 0.0 && budget_scale <= 16.0),
                "budget_scale must be 0 (default) or in (0, 16]");
        if (enable) dd_alloc(m);
        m->dd_on = enable != 0;
        m->dd_scale = budget_scale > 0.0 ? budget_scale : 1.05;
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_destroy(rafem_mesh mesh) {
    return guard([&]() -> rafem_status {
        free_mesh(mesh);
        return RAFEM_OK;
    });
}

rafem_status rafem_mesh_get_stats(rafem_mesh m, rafem_mesh_stats* out) {
    return guard([&]() -> rafem_status {
        require(m != nullptr && out != nullptr, "NULL argument");
        out->n_nodes = m->n;
        out->n_elems = m->E;
        out->nnz = m->nnz;
        out->n_dirichlet = m->nD;
        out->nodes_per_elem = m->npe;
        out->n_colours = m->n_colours;
        out->n_samples = m->S;
        out->slabs_per_block = m->spmv.slabs_per_block;
        out->slabs_per_block32 = m->spmv32.slabs_per_block;
        out->int16_columns = m->sdel ? 1 : 0;
        out->shared_offset_slabs = m->shared_slabs;
        out->slabs = m->nslabs;
        out->row_assembly = m->row_asm ? 1 : 0;
        out->max_row_entries = m->max_w;
        out->value_slots = m->sell_nnz;
        out->index_bytes = m->index_bytes;
        out->device_driven = m->dd_on ? 1 : 0;
        out->tuned_from_cache = m->tuned_from_cache ? 1 : 0;
        out->device_driven_solves = m->dd_solves;
        out->device_driven_redone = m->dd_redone;
        out->int32_column_slabs = m->int32_slabs;
        out->streamed_values = m->spmv.stream;
        out->streamed_values32 = m->spmv32.stream;
        out->resident_slots = m->spmv.stream ? m->spmv.resident : 0;
        out->resident_slots32 = m->spmv32.stream ? m->spmv32.resident : 0;
        out->launch_bound = m->spmv.min_blocks;
        out->launch_bound32 = m->spmv32.min_blocks;
        return RAFEM_OK;
    });
}

rafem_status rafem_assemble_csr(rafem_mesh m, const double* mass_coef_d, const double* stiff_coef_d,
                                const double* dir_vals_d, int32_t* row_ptr_d, int32_t* col_idx_d,
                                double* vals_d, float* vals32_d, double* rhs_lift_d,
                                void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(vals_d != nullptr, "vals is NULL");
        require(dir_vals_d == nullptr || rhs_lift_d != nullptr, "rhs_lift is required with dir_vals");
        require(dir_vals_d == nullptr || m->nD > 0, "dir_vals given but the mesh has no Dirichlet nodes");
        hipStream_t s = (hipStream_t)stream;
        if (row_ptr_d)
            RAFEM_HIP(hipMemcpyAsync(row_ptr_d, m->rp, (m->n + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (col_idx_d)
            RAFEM_HIP(hipMemcpyAsync(col_idx_d, m->ci, m->nnz * 4, hipMemcpyDeviceToDevice, s));
        const Layout L = csr_layout(m);
        assemble_into(m, L, m->nnz, mass_coef_d, stiff_coef_d, vals_d, s);
        const int do_lift = dir_vals_d != nullptr;
        if (do_lift) launch_scatter_dirichlet(m->dir_ids, dir_vals_d, m->nD, m->gtmp, s);
        if (do_lift || vals32_d)
            launch_lift((int)m->n, L, vals_d, vals32_d, m->isD, m->gtmp,
                        do_lift ? rhs_lift_d : nullptr, nullptr, nullptr, do_lift, s);
        RAFEM_HIP(hipGetLastError());
        return RAFEM_OK;
    });
}

rafem_status rafem_solve(rafem_mesh m, const int32_t* row_ptr_d, const int32_t* col_idx_d,
                         const double* vals_d, const float* vals32_d, const double* b_d,
                         double* x_d, const rafem_solve_opts* opts, rafem_solve_info* info,
                         void* stream) {
    rafem_status st = RAFEM_OK;
    rafem_status rc = guard([&]() -> rafem_status {
        check_device(m);
        require(row_ptr_d && col_idx_d && vals_d && b_d && x_d, "NULL matrix or vector argument");
        SolveOpts o = resolve_opts(opts, 1e-10);
        require(o.precision != RAFEM_MIXED || vals32_d != nullptr, "MIXED precision needs vals32");
        hipStream_t s = (hipStream_t)stream;
        const Mat A = csr_matrix(m, row_ptr_d, col_idx_d, vals_d, vals32_d);
        if (o.precision == RAFEM_MIXED)
            st = pcg_mixed(m, A, whole_mesh(m), nullptr, nullptr, b_d, x_d, o, info, s, nullptr);
        else
            st = pcg64(m, A, whole_mesh(m), nullptr, b_d, x_d, o, info, s, nullptr);
        if (st != RAFEM_OK)
            set_error(st == RAFEM_E_NOCONV ? "iteration limit reached" : "PCG breakdown (p.Ap <= 0 or non-finite)");
        return st;
    });
    return rc;
}

rafem_status rafem_solve_enqueue(rafem_mesh m, const int32_t* row_ptr_d,
                                 const int32_t* col_idx_d, const double* vals_d,
                                 const float* vals32_d, const double* b_d, double* x_d,
                                 const rafem_solve_opts* opts, int32_t iterations,
                                 int32_t refinements, rafem_device_info* info_d, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(m->S == 1, "rafem_solve_enqueue runs on single-mesh handles");
        require(row_ptr_d && col_idx_d && vals_d && b_d && x_d && info_d,
                "NULL matrix, vector or info argument");
        SolveOpts o = resolve_opts(opts, 1e-10);
        require(o.precision != RAFEM_MIXED || vals32_d != nullptr, "MIXED precision needs vals32");
        require(iterations >= 1 && iterations <= 100000, "iterations must be in [1, 100000]");
        require(o.precision != RAFEM_MIXED || (refinements >= 1 && refinements < kDdMaxRounds),
                "refinements must be in [1, 14]");
        hipStream_t s = (hipStream_t)stream;
        const Mat A = csr_matrix(m, row_ptr_d, col_idx_d, vals_d, vals32_d);
        solve_enqueue(m, A, whole_mesh(m), b_d, x_d, o, iterations, refinements, info_d, s);
        return RAFEM_OK;
    });
}

rafem_status rafem_solve_adjoint(rafem_mesh m, const int32_t* row_ptr_d, const int32_t* col_idx_d,
                                 const double* vals_d, const float* vals32_d, const double* g_d,
                                 double* lambda_d, const rafem_solve_opts* opts,
                                 rafem_solve_info* info, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(row_ptr_d && col_idx_d && vals_d && g_d && lambda_d, "NULL matrix or vector argument");
        SolveOpts o = resolve_opts(opts, 1e-10);
        require(o.precision != RAFEM_MIXED || vals32_d != nullptr, "MIXED precision needs vals32");
        hipStream_t s = (hipStream_t)stream;
        // right-hand side with Dirichlet rows zeroed; the adjoint of a prescribed value is 0
        RAFEM_HIP(hipMemcpyAsync(m->bT, g_d, m->n * 8, hipMemcpyDeviceToDevice, s));
        launch_fill(m->gtmp, m->n, 0.0, s);
        launch_set_dirichlet(m->dir_ids, m->gtmp, m->nD, m->bT, s);
        launch_set_dirichlet(m->dir_ids, m->gtmp, m->nD, lambda_d, s);
        const Mat A = csr_matrix(m, row_ptr_d, col_idx_d, vals_d, vals32_d);
        rafem_status st;
        if (o.precision == RAFEM_MIXED)
            st = pcg_mixed(m, A, whole_mesh(m), nullptr, nullptr, m->bT, lambda_d, o, info, s,
                           nullptr);
        else
            st = pcg64(m, A, whole_mesh(m), nullptr, m->bT, lambda_d, o, info, s, nullptr);
        if (st != RAFEM_OK)
            set_error(st == RAFEM_E_NOCONV ? "iteration limit reached" : "PCG breakdown (p.Ap <= 0 or non-finite)");
        return st;
    });
}

rafem_status rafem_spmv(rafem_mesh m, const int32_t* row_ptr_d, const int32_t* col_idx_d,
                        const double* vals_d, const double* x_d, double* y_d,
                        const float* vals32_d, const float* x32_d, float* y32_d, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(row_ptr_d && col_idx_d, "NULL structure");
        hipStream_t s = (hipStream_t)stream;
        if (vals_d) {
            require(x_d && y_d, "NULL x or y");
            launch_spmv64(csr_matrix(m, row_ptr_d, col_idx_d, vals_d, nullptr), m->spmv, x_d, y_d, s);
        } else {
            require(vals32_d && x32_d && y32_d, "NULL FP32 arguments");
            launch_spmv32(csr_matrix(m, row_ptr_d, col_idx_d, nullptr, vals32_d), m->spmv, x32_d, y32_d,
                          s);
        }
        RAFEM_HIP(hipGetLastError());
        return RAFEM_OK;
    });
}

rafem_status rafem_spmv_step(rafem_mesh m, int32_t matrix, int32_t precision, const void* x_d,
                             void* y_d, const double* b_d, double* dots_h, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(matrix == 0 || matrix == 1, "matrix must be 0 (potential) or 1 (bioheat)");
        require(precision == RAFEM_FP64 || precision == RAFEM_MIXED, "precision");
        require(x_d && y_d, "NULL x or y");
        require(!b_d || precision == RAFEM_FP64, "the residual form (b given) is FP64 only");
        if (matrix == 0 && !m->potential_ready)
            throw Error{RAFEM_E_STATE, "no step has assembled the potential matrix yet"};
        if (matrix == 1 && !m->bioheat_ready)
            throw Error{RAFEM_E_STATE, "no step has assembled the bioheat matrix yet"};
        hipStream_t s = (hipStream_t)stream;
        const bool fp32 = precision == RAFEM_MIXED;
        const Mat A = matrix == 0 ? step_matrix(m, m->valsV, m->valsV32)
                                  : step_matrix(m, m->valsT, m->valsT32);
        const int S = m->S;
        const Samples smp = step_samples(m);
        PcgState* chk = m->st + 2 * S;
        launch_state_init(chk, S, 0.0, 0, nullptr, s);  // done = 0: no sample is skipped
        if (b_d) {
            launch_residual64(A, m->spmv, b_d, (const double*)x_d, (double*)y_d, m->partials, chk,
                              smp, 0, s);
            RAFEM_HIP(hipGetLastError());
            if (dots_h) {
                std::vector<PcgState> h(S);
                RAFEM_HIP(hipMemcpyAsync(h.data(), chk, S * sizeof(PcgState),
                                         hipMemcpyDeviceToHost, s));
                RAFEM_HIP(hipStreamSynchronize(s));
                for (int q = 0; q < S; ++q) {
                    dots_h[2 * q] = h[q].rr;
                    dots_h[2 * q + 1] = h[q].bb;
                }
            }
            return RAFEM_OK;
        }
        const GridInfo g =
            fp32 ? launch_spmv_dot32(A, m->spmv32, (const float*)x_d, (float*)y_d, m->part_pq,
                                     chk, smp, s)
                 : launch_spmv_dot64(A, m->spmv, (const double*)x_d, (double*)y_d, m->part_pq,
                                     chk, smp, s);
        RAFEM_HIP(hipGetLastError());
        if (dots_h) {
            // the kernel's own per-group partials of x.(A x), added per sample in slot order
            std::vector<double> part(std::max(g.nb, 1));
            RAFEM_HIP(hipMemcpyAsync(part.data(), m->part_pq, g.nb * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
            RAFEM_HIP(hipStreamSynchronize(s));
            for (int q = 0; q < S; ++q) {
                const int64_t b0 = m->node_off[q] / g.rpb;
                const int64_t b1 = std::min<int64_t>((m->node_off[q + 1] + g.rpb - 1) / g.rpb, g.nb);
                double t = 0.0;
                for (int64_t k = b0; k < b1; ++k) t += part[k];
                dots_h[q] = t;
            }
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_spmv_timing(rafem_mesh m, int32_t precision, int32_t n_copies, int32_t reps,
                               double* mean_us) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(precision == RAFEM_FP64 || precision == RAFEM_MIXED, "precision");
        require(n_copies >= 1 && n_copies <= 64 && reps >= 1 && reps <= 100000 && mean_us,
                "n_copies in [1, 64], reps in [1, 100000], mean_us");
        if (!m->potential_ready) throw Error{RAFEM_E_STATE, "no step has assembled the matrix yet"};
        const bool fp32 = precision == RAFEM_MIXED;
        const size_t bytes = (size_t)m->sell_nnz * (fp32 ? sizeof(float) : sizeof(double));
        std::vector<void*> copies(n_copies, nullptr);
        std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
        auto release = [&]() {
            for (void* c : copies)
                if (c) (void)hipFree(c);
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
        };
        try {
            for (auto& c : copies) {
                if (hipMalloc(&c, bytes) != hipSuccess) {
                    (void)hipGetLastError();
                    c = nullptr;
                    throw Error{RAFEM_E_NOMEM, "value copies do not fit in device memory"};
                }
                RAFEM_HIP(hipMemcpy(c, fp32 ? (const void*)m->valsV32 : (const void*)m->valsV,
                                    bytes, hipMemcpyDeviceToDevice));
            }
            for (auto& e : ev) RAFEM_HIP(hipEventCreate(&e));
            hipStream_t s = nullptr;
            const int S = m->S;
            Samples smp{S, m->row_off, m->row_tab};
            PcgState* chk = m->st + 2 * S;
            launch_state_init(chk, S, 0.0, 0, nullptr, s);
            launch_fill(m->p, m->n, 1.0, s);
            launch_fill32(m->p32, m->n, 1.0f, s);
            for (int r = 0; r < reps; ++r) {
                Mat A = step_matrix(m, fp32 ? nullptr : (const double*)copies[r % n_copies],
                                    fp32 ? (const float*)copies[r % n_copies] : nullptr);
                if (fp32)
                    launch_spmv_dot32(A, m->spmv32, m->p32, m->q32, m->part_pq, chk, smp, s,
                                      ev[2 * r], ev[2 * r + 1]);
                else
                    launch_spmv_dot64(A, m->spmv, m->p, m->q, m->part_pq, chk, smp, s, ev[2 * r],
                                      ev[2 * r + 1]);
            }
            RAFEM_HIP(hipGetLastError());
            RAFEM_HIP(hipStreamSynchronize(s));
            double sum = 0.0;
            for (int r = 0; r < reps; ++r) {
                float ms = 0.f;
                RAFEM_HIP(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
                sum += 1000.0 * ms;
            }
            *mean_us = sum / reps;
        } catch (...) {
            release();
            throw;
        }
        release();
        return RAFEM_OK;
    });
}

rafem_status rafem_profile_enable(rafem_mesh m, int32_t enable) {
    return guard([&]() -> rafem_status {
        check_device(m);
        if (enable && !m->prof_on) {
            m->prof_ev.resize(2 * kProfCap);
            for (auto& e : m->prof_ev) e = nullptr;
            for (auto& e : m->prof_ev) {
                if (hipEventCreate(&e) != hipSuccess) {
                    e = nullptr;
                    profile_off(m);
                    throw Error{RAFEM_E_HIP, "hipEventCreate failed"};
                }
            }
            m->prof_on = true;
        } else if (!enable && m->prof_on) {
            RAFEM_HIP(hipDeviceSynchronize());
            profile_off(m);
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_regions_enable(rafem_mesh m, int32_t enable) {
    return guard([&]() -> rafem_status {
        check_device(m);
        if (enable) {
            m->reg_on = true;
            m->reg_kind.clear();
        } else {
            RAFEM_HIP(hipDeviceSynchronize());
            regions_off(m);
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_regions_read(rafem_mesh m, rafem_regions* out, int32_t reset) {
    return guard([&]() -> rafem_status {
        require(m != nullptr && out != nullptr, "NULL argument");
        out->assembly_ms = m->reg_ms[kRegAssembly];
        out->solve_ms = m->reg_ms[kRegSolve];
        out->check_ms = m->reg_ms[kRegCheck];
        out->steps = m->reg_steps;
        if (reset) {
            m->reg_ms[0] = m->reg_ms[1] = m->reg_ms[2] = 0.0;
            m->reg_steps = 0;
        }
        return RAFEM_OK;
    });
}

rafem_status rafem_profile_read(rafem_mesh m, int32_t precision, double* mean_us, int64_t* count,
                                int32_t reset) {
    return guard([&]() -> rafem_status {
        require(m != nullptr, "mesh is NULL");
        require(precision == RAFEM_FP64 || precision == RAFEM_MIXED, "bad precision");
        const int k = precision == RAFEM_MIXED ? 1 : 0;
        if (mean_us) *mean_us = m->prof_cnt[k] ? m->prof_sum_us[k] / (double)m->prof_cnt[k] : 0.0;
        if (count) *count = m->prof_cnt[k];
        if (reset) {
            m->prof_sum_us[k] = 0.0;
            m->prof_cnt[k] = 0;
        }
        return RAFEM_OK;
    });
}

namespace {

void check_step_args(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                     const double* perf_e_d, const double* sigma0_e_d, const double* dir_V_d,
                     const double* dir_T_d, const double* T_d, const double* V_d) {
    check_device(m);
    require(phys != nullptr, "phys is NULL");
    require(k_e_d && perf_e_d && T_d, "NULL k, perfusion or T");
    require(m->nD == 0 || dir_T_d != nullptr, "dir_T is NULL");
    require(phys->dt > 0.0 && std::isfinite(phys->dt), "dt must be > 0");
    require(std::isfinite(phys->rho_c) && std::isfinite(phys->T_a), "non-finite physics constant");
    if (phys->coupled) {
        require(sigma0_e_d && V_d, "coupled step needs sigma0 and V");
        require(m->nD == 0 || dir_V_d != nullptr, "dir_V is NULL");
    }
}

// The body of one coupled step: sigma from T_sig, the bioheat right-hand side from T_rhs
// (T^n), T_out in: initial guess, out: T^{n+1} (may alias T_rhs and T_sig), V in/out.
// reuse_bioheat: the bioheat matrix of this dt is already assembled.
rafem_status step_core(rafem_mesh m, const rafem_phys* phys, bool reuse_bioheat,
                       const double* k_e_d, const double* perf_e_d, const double* sigma0_e_d,
                       const double* dir_V_d, const double* dir_T_d, const double* T_sig,
                       const double* T_rhs, double* T_out, double* V_d, const SolveOpts& o,
                       rafem_step_info& inf, hipStream_t s) {
    const bool mixed = o.precision == RAFEM_MIXED;
    region_mark(m, kRegAssembly, s);
    launch_scatter_dirichlet(m->dir_ids, dir_T_d, m->nD, m->gT, s);
    if (!reuse_bioheat) assemble_bioheat(m, phys, k_e_d, perf_e_d, s);
    if (phys->coupled) {
        launch_scatter_dirichlet(m->dir_ids, dir_V_d, m->nD, m->gV, s);
        assemble_potential(m, phys, sigma0_e_d, T_sig, s);
        launch_set_dirichlet(m->dir_ids, m->gV, m->nD, V_d, s);
        RAFEM_HIP(hipGetLastError());
        const Mat AV = step_matrix(m, m->valsV, m->valsV32);
        if (!m->tuned) autotune_spmv(m, AV, s);
        region_mark(m, kRegSolve, s);
        solve_step(m, o, AV, m->dinvV, m->dinvV32, m->liftV, V_d, &inf.V, s, kSolvePotential);
        region_mark(m, kRegAssembly, s);
        if (inf.V.status != RAFEM_OK) {
            set_error("potential solve failed");
            return inf.V.status;
        }
    }
    if (m->row_asm) {
        launch_bioheat_rhs_rows(m->npe, m->affine, m->E, m->conn, m->xyz, m->geo, T_rhs,
                                phys->coupled ? V_d : nullptr, m->sigma, perf_e_d,
                                phys->rho_c / phys->dt, phys->T_a, phys->coupled ? 1 : 0, m->erhs,
                                (int)m->n, m->isptr, m->n2e, m->liftT, m->isD, m->bT, s);
    } else {
        launch_fill(m->rhs, m->n, 0.0, s);
        for (int c = 0; c < m->n_colours; ++c) {
            const int off = m->colour_off[c], cnt = m->colour_off[c + 1] - off;
            launch_bioheat_rhs_colour(m->npe, m->affine, m->colour_elems + off, cnt, m->conn,
                                      m->xyz, T_rhs, phys->coupled ? V_d : nullptr, m->sigma,
                                      perf_e_d, phys->rho_c / phys->dt, phys->T_a,
                                      phys->coupled ? 1 : 0, m->rhs, s);
        }
        launch_finish_rhs((int)m->n, m->rhs, m->liftT, m->isD, m->bT, s);
    }
    launch_set_dirichlet(m->dir_ids, m->gT, m->nD, T_out, s);
    RAFEM_HIP(hipGetLastError());
    const Mat AT = step_matrix(m, m->valsT, m->valsT32);
    if (!m->tuned) autotune_spmv(m, AT, s);
    region_mark(m, kRegSolve, s);
    solve_step(m, o, AT, m->dinvT, m->dinvT32, m->bT, T_out, &inf.T, s, kSolveBioheat);
    region_mark(m, kRegCheck, s);
    if (inf.T.status != RAFEM_OK) {
        set_error("bioheat solve failed");
        return inf.T.status;
    }
    return RAFEM_OK;
}

}  // namespace

rafem_status rafem_step(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                        const double* perf_e_d, const double* sigma0_e_d, const double* dir_V_d,
                        const double* dir_T_d, double* T_d, double* V_d,
                        const rafem_solve_opts* opts, rafem_step_info* info, void* stream) {
    return guard([&]() -> rafem_status {
        check_step_args(m, phys, k_e_d, perf_e_d, sigma0_e_d, dir_V_d, dir_T_d, T_d, V_d);
        if (phys->reuse_bioheat && !m->bioheat_ready)
            throw Error{RAFEM_E_STATE, "reuse_bioheat set but no bioheat matrix has been assembled"};
        const SolveOpts o = resolve_opts(opts, 1e-12);
        rafem_step_info local{};
        rafem_step_info& inf = info ? *info : local;
        std::memset(&inf, 0, sizeof(inf));
        // a bioheat matrix built for another time step is rebuilt
        const bool reuse = phys->reuse_bioheat && m->bioheat_dt == phys->dt;
        hipStream_t s = (hipStream_t)stream;
        region_begin(m);
        if (phys->extrapolate < 0 || phys->extrapolate > 2)
            throw Error{RAFEM_E_ARG, "phys.extrapolate must be 0, 1 or 2"};
        if (phys->extrapolate_order < 0 || phys->extrapolate_order > rafem_mesh_s::kXgSlots - 1)
            throw Error{RAFEM_E_ARG, "phys.extrapolate_order must be in [0, 4]"};
        if (!phys->extrapolate) {
            m->xg_kept = 0;
            m->step_q = -1;
            const rafem_status st = step_core(m, phys, reuse, k_e_d, perf_e_d, sigma0_e_d,
                                              dir_V_d, dir_T_d, T_d, T_d, T_d, V_d, o, inf, s);
            region_flush(m, s);
            return st;
        }
        // keep (T^n, V^n) in slot xg_cur; start the solves from the polynomial through it and
        // the kept earlier states (at most `order` of them), taken at t_n + dt
        if (phys->extrapolate == 2) m->xg_kept = 0;
        const int order = std::max(1, phys->extrapolate_order);
        const int K = rafem_mesh_s::kXgSlots;
        const size_t bytes = (size_t)m->n * sizeof(double);
        const int cur = m->xg_cur;
        double* Tn = m->xg_T[cur];
        double* Vn = m->xg_V[cur];
        region_mark(m, kRegCheck, s);
        RAFEM_HIP(hipMemcpyAsync(Tn, T_d, bytes, hipMemcpyDeviceToDevice, s));
        if (phys->coupled) RAFEM_HIP(hipMemcpyAsync(Vn, V_d, bytes, hipMemcpyDeviceToDevice, s));
        const int q = std::min(order, m->xg_kept);
        m->step_q = q;
        if (q == 1) {
            const double c = phys->dt / m->xg_h[0];
            const int p1 = (cur + K - 1) % K;
            launch_extrapolate((int)m->n, Tn, m->xg_T[p1], c, T_d, s);
            if (phys->coupled) launch_extrapolate((int)m->n, Vn, m->xg_V[p1], c, V_d, s);
        } else if (q >= 2) {
            // Lagrange weights of the nodes t_k = t_n - (h_1 + ... + h_k), k = 0 .. q
            double t[rafem_mesh_s::kXgSlots] = {}, w[rafem_mesh_s::kXgSlots];
            for (int k = 1; k <= q; ++k) t[k] = t[k - 1] - m->xg_h[k - 1];
            for (int i = 0; i <= q; ++i) {
                w[i] = 1.0;
                for (int k = 0; k <= q; ++k)
                    if (k != i) w[i] *= (phys->dt - t[k]) / (t[i] - t[k]);
            }
            const double* xT[rafem_mesh_s::kXgSlots];
            const double* xV[rafem_mesh_s::kXgSlots];
            for (int k = 0; k <= q; ++k) {
                xT[k] = m->xg_T[(cur + K - k) % K];
                xV[k] = m->xg_V[(cur + K - k) % K];
            }
            launch_extrapolate_poly((int)m->n, q + 1, xT, w, T_d, s);
            if (phys->coupled) launch_extrapolate_poly((int)m->n, q + 1, xV, w, V_d, s);
        }
        const rafem_status st = step_core(m, phys, reuse, k_e_d, perf_e_d, sigma0_e_d, dir_V_d,
                                          dir_T_d, Tn, Tn, T_d, V_d, o, inf, s);
        if (st == RAFEM_OK && phys->coupled) {
            m->xg_kept = std::min(m->xg_kept + 1, K - 1);
            for (int k = K - 2; k > 0; --k) m->xg_h[k] = m->xg_h[k - 1];
            m->xg_h[0] = phys->dt;
        } else {
            m->xg_kept = 0;
        }
        m->xg_cur = (cur + 1) % K;
        region_flush(m, s);
        return st;
    });
}

rafem_status rafem_step_pc(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                           const double* perf_e_d, const double* sigma0_e_d,
                           const double* dir_V_d, const double* dir_T_d, const double* T_prev_d,
                           double dt_prev, double* T_d, double* V_d, const rafem_solve_opts* opts,
                           const rafem_corrector_opts* copts, rafem_corrector_info* info,
                           void* stream) {
    return guard([&]() -> rafem_status {
        check_step_args(m, phys, k_e_d, perf_e_d, sigma0_e_d, dir_V_d, dir_T_d, T_d, V_d);
        require(m->S == 1, "the predictor-corrector step runs on single meshes");
        m->step_q = -2;
        require(!T_prev_d || (dt_prev > 0.0 && std::isfinite(dt_prev)),
                "dt_prev must be > 0 when T_prev is given");
        const double eps = copts && copts->tol > 0.0 ? copts->tol : 1e-10;
        const int max_iters = copts && copts->max_iters > 0 ? copts->max_iters : 50;
        require(std::isfinite(eps) && eps < 1.0, "corrector tol must be in (0, 1)");
        const SolveOpts o = resolve_opts(opts, 1e-12);
        hipStream_t s = (hipStream_t)stream;
        rafem_corrector_info local{};
        rafem_corrector_info& ci = info ? *info : local;
        std::memset(&ci, 0, sizeof(ci));
        const size_t bytes = (size_t)m->n * sizeof(double);
        m->xg_kept = 0;
        region_begin(m);
        region_mark(m, kRegCheck, s);
        // keep (T^n, V^n) to restore a rejected step; predictor into pc_Tk
        RAFEM_HIP(hipMemcpyAsync(m->pc_Tn, T_d, bytes, hipMemcpyDeviceToDevice, s));
        if (phys->coupled)
            RAFEM_HIP(hipMemcpyAsync(m->pc_Vn, V_d, bytes, hipMemcpyDeviceToDevice, s));
        launch_extrapolate((int)m->n, m->pc_Tn, T_prev_d, T_prev_d ? phys->dt / dt_prev : 0.0,
                           m->pc_Tk, s);
        bool reuse = phys->reuse_bioheat && m->bioheat_ready && m->bioheat_dt == phys->dt;
        rafem_status st = RAFEM_OK;
        for (int k = 1; k <= max_iters; ++k) {
            RAFEM_HIP(hipMemcpyAsync(T_d, m->pc_Tk, bytes, hipMemcpyDeviceToDevice, s));
            rafem_step_info inf{};
            st = step_core(m, phys, reuse, k_e_d, perf_e_d, sigma0_e_d, dir_V_d, dir_T_d,
                           m->pc_Tk, m->pc_Tn, T_d, V_d, o, inf, s);
            reuse = true;
            ci.iters = k;
            ci.solver_iters += inf.V.iters + inf.T.iters;
            if (st != RAFEM_OK) break;
            // relative change of T over this corrector iteration
            double h[2];
            launch_change_norm((int)m->n, T_d, m->pc_Tk, m->partials, m->pc_norm, s);
            RAFEM_HIP(hipMemcpyAsync(h, m->pc_norm, sizeof(h), hipMemcpyDeviceToHost, s));
            RAFEM_HIP(hipStreamSynchronize(s));
            ci.change = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
            RAFEM_HIP(hipMemcpyAsync(m->pc_Tk, T_d, bytes, hipMemcpyDeviceToDevice, s));
            if (!std::isfinite(ci.change)) {
                st = RAFEM_E_BREAKDOWN;
                set_error("non-finite temperature change in the corrector");
                break;
            }
            if (ci.change <= eps) {
                ci.accepted = 1;
                break;
            }
        }
        ci.status = st;
        if (!ci.accepted) {  // rejected (or failed): leave (T^n, V^n) as they were
            RAFEM_HIP(hipMemcpyAsync(T_d, m->pc_Tn, bytes, hipMemcpyDeviceToDevice, s));
            if (phys->coupled)
                RAFEM_HIP(hipMemcpyAsync(V_d, m->pc_Vn, bytes, hipMemcpyDeviceToDevice, s));
            RAFEM_HIP(hipStreamSynchronize(s));
        }
        region_flush(m, s);
        return st;
    });
}

namespace {

void check_mono_args(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                     const double* perf_e_d, const double* sigma0_e_d, const double* T_n_d,
                     const double* T_d, const double* V_d) {
    check_device(m);
    require(m->S == 1, "the monolithic corrector runs on single meshes");
    require(phys != nullptr, "phys is NULL");
    require(phys->coupled != 0, "the monolithic corrector needs a coupled problem");
    require(k_e_d && perf_e_d && sigma0_e_d, "NULL k, perfusion or sigma0");
    require(T_n_d && T_d && V_d, "NULL T^n, T or V");
    require(phys->dt > 0.0 && std::isfinite(phys->dt), "dt must be > 0");
    require(std::isfinite(phys->rho_c) && std::isfinite(phys->T_a) &&
                std::isfinite(phys->alpha_sigma) && std::isfinite(phys->T_ref),
            "non-finite physics constant");
}

}  // namespace

rafem_status rafem_mono_jacobian(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                                 const double* perf_e_d, const double* sigma0_e_d,
                                 const double* T_n_d, const double* T_d, const double* V_d,
                                 double* planes_d, double* R_d, void* stream) {
    return guard([&]() -> rafem_status {
        check_mono_args(m, phys, k_e_d, perf_e_d, sigma0_e_d, T_n_d, T_d, V_d);
        require(planes_d && R_d, "NULL output");
        hipStream_t s = (hipStream_t)stream;
        mono_export(m, phys, k_e_d, perf_e_d, sigma0_e_d, T_n_d, T_d, V_d, planes_d, R_d, s);
        RAFEM_HIP(hipStreamSynchronize(s));
        return RAFEM_OK;
    });
}

rafem_status rafem_mono_solve(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                              const double* perf_e_d, const double* sigma0_e_d,
                              const double* T_n_d, const double* T_d, const double* V_d,
                              const rafem_gmres_opts* opts, double* delta_d, double* hist_d,
                              int32_t hist_len, rafem_gmres_info* info, void* stream) {
    return guard([&]() -> rafem_status {
        check_mono_args(m, phys, k_e_d, perf_e_d, sigma0_e_d, T_n_d, T_d, V_d);
        require(delta_d != nullptr, "delta is NULL");
        require(hist_len >= 0 && (hist_len == 0 || hist_d), "bad residual history buffer");
        const GmresOpts o = resolve_gmres(opts);
        hipStream_t s = (hipStream_t)stream;
        mono_ensure(m, o.m, o.precision == RAFEM_MIXED);
        mono_assemble(m, phys, k_e_d, perf_e_d, sigma0_e_d, T_n_d, T_d, V_d, s);
        rafem_gmres_info local{};
        const rafem_status st = gmres_solve(m, m->mono_rhs, delta_d, o, hist_len ? hist_d : nullptr,
                                            hist_len, info ? info : &local, s);
        if (st != RAFEM_OK) set_error("GMRES did not converge");
        return st;
    });
}

rafem_status rafem_step_mono(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                             const double* perf_e_d, const double* sigma0_e_d,
                             const double* dir_V_d, const double* dir_T_d,
                             const double* T_prev_d, double dt_prev, double* T_d, double* V_d,
                             const rafem_gmres_opts* opts, const rafem_corrector_opts* copts,
                             rafem_mono_info* info, void* stream) {
    return guard([&]() -> rafem_status {
        check_mono_args(m, phys, k_e_d, perf_e_d, sigma0_e_d, T_d, T_d, V_d);
        m->step_q = -2;
        require(m->nD == 0 || (dir_V_d && dir_T_d), "dir_V or dir_T is NULL");
        require(!T_prev_d || (dt_prev > 0.0 && std::isfinite(dt_prev)),
                "dt_prev must be > 0 when T_prev is given");
        const double eps = copts && copts->tol > 0.0 ? copts->tol : 1e-10;
        const int max_iters = copts && copts->max_iters > 0 ? copts->max_iters : 50;
        require(std::isfinite(eps) && eps < 1.0, "corrector tol must be in (0, 1)");
        const GmresOpts o = resolve_gmres(opts);
        hipStream_t s = (hipStream_t)stream;
        rafem_mono_info local{};
        rafem_mono_info& mi = info ? *info : local;
        std::memset(&mi, 0, sizeof(mi));
        mono_ensure(m, o.m, o.precision == RAFEM_MIXED);
        const size_t bytes = (size_t)m->n * sizeof(double);
        m->xg_kept = 0;
        region_begin(m);
        region_mark(m, kRegCheck, s);
        // keep (T^n, V^n) to restore a rejected step; the iterate starts at (T*, V^n) with
        // the Dirichlet values
        RAFEM_HIP(hipMemcpyAsync(m->pc_Tn, T_d, bytes, hipMemcpyDeviceToDevice, s));
        RAFEM_HIP(hipMemcpyAsync(m->pc_Vn, V_d, bytes, hipMemcpyDeviceToDevice, s));
        launch_extrapolate((int)m->n, m->pc_Tn, T_prev_d, T_prev_d ? phys->dt / dt_prev : 0.0,
                           T_d, s);
        launch_scatter_dirichlet(m->dir_ids, dir_T_d, m->nD, m->gT, s);
        launch_scatter_dirichlet(m->dir_ids, dir_V_d, m->nD, m->gV, s);
        launch_set_dirichlet(m->dir_ids, m->gT, m->nD, T_d, s);
        launch_set_dirichlet(m->dir_ids, m->gV, m->nD, V_d, s);
        rafem_status st = RAFEM_OK;
        for (int k = 1; k <= max_iters; ++k) {
            region_mark(m, kRegAssembly, s);
            mono_assemble(m, phys, k_e_d, perf_e_d, sigma0_e_d, m->pc_Tn, T_d, V_d, s);
            rafem_gmres_info gi{};
            region_mark(m, kRegSolve, s);
            st = gmres_solve(m, m->mono_rhs, m->mono_delta, o, nullptr, 0, &gi, s);
            region_mark(m, kRegCheck, s);
            mi.iters = k;
            mi.gmres_iters += gi.iters;
            mi.gmres_cycles += gi.cycles;
            mi.relres_true_max = std::max(mi.relres_true_max, gi.relres_true);
            if (st != RAFEM_OK) {
                set_error("GMRES did not converge in the monolithic corrector");
                break;
            }
            double h[2];
            launch_newton_apply((int)m->n, m->mono_delta, T_d, V_d, m->gm_part, m->pc_norm, s);
            RAFEM_HIP(hipMemcpyAsync(h, m->pc_norm, sizeof(h), hipMemcpyDeviceToHost, s));
            RAFEM_HIP(hipStreamSynchronize(s));
            mi.change = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
            if (!std::isfinite(mi.change)) {
                st = RAFEM_E_BREAKDOWN;
                set_error("non-finite temperature change in the monolithic corrector");
                break;
            }
            if (mi.change <= eps) {
                mi.accepted = 1;
                break;
            }
        }
        mi.status = st;
        if (!mi.accepted) {
            RAFEM_HIP(hipMemcpyAsync(T_d, m->pc_Tn, bytes, hipMemcpyDeviceToDevice, s));
            RAFEM_HIP(hipMemcpyAsync(V_d, m->pc_Vn, bytes, hipMemcpyDeviceToDevice, s));
            RAFEM_HIP(hipStreamSynchronize(s));
        }
        region_flush(m, s);
        return st;
    });
}

rafem_status rafem_step_vjp(rafem_mesh m, const rafem_phys* phys, const double* k_e_d,
                            const double* perf_e_d, const double* sigma0_e_d,
                            const double* dir_V_d, const double* dir_T_d, const double* T_prev_d,
                            const double* V_d, const double* T_d, double* lambda_d,
                            double* grad_k_d, double* grad_perf_d, const rafem_solve_opts* opts,
                            rafem_step_info* info, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(phys != nullptr, "phys is NULL");
        require(k_e_d && perf_e_d && T_d && lambda_d && grad_k_d && grad_perf_d,
                "NULL k, perfusion, T, lambda or gradient");
        m->step_q = -2;
        require(m->nD == 0 || dir_T_d != nullptr, "dir_T is NULL");
        require(phys->dt > 0.0 && std::isfinite(phys->dt), "dt must be > 0");
        if (phys->coupled) {
            require(sigma0_e_d && V_d && T_prev_d, "coupled reverse step needs sigma0, V and T_prev");
            require(m->nD == 0 || dir_V_d != nullptr, "dir_V is NULL");
        }
        if (phys->reuse_bioheat && !m->bioheat_ready)
            throw Error{RAFEM_E_STATE, "reuse_bioheat set but no bioheat matrix has been assembled"};
        if (phys->extrapolate < 0 || phys->extrapolate > 2)
            throw Error{RAFEM_E_ARG, "phys.extrapolate must be 0, 1 or 2"};
        SolveOpts o = resolve_opts(opts, 1e-12);
        hipStream_t s = (hipStream_t)stream;
        rafem_step_info local{};
        rafem_step_info& inf = info ? *info : local;
        std::memset(&inf, 0, sizeof(inf));
        const int npe = m->npe, aff = m->affine;
        // adjoint solves of a reverse sweep start from the previous call's mu and nu (the
        // adjoint states of the step after), else from zero
        const bool warm = phys->extrapolate == 1 && m->adj_kept;
        const bool warm_nu = warm && m->adj_kept_nu;
        m->adj_kept = false;

        launch_scatter_dirichlet(m->dir_ids, dir_T_d, m->nD, m->gT, s);
        if (!phys->reuse_bioheat || m->bioheat_dt != phys->dt)
            assemble_bioheat(m, phys, k_e_d, perf_e_d, s);
        // mu: A_T mu = lambda with the Dirichlet rows of the load zeroed
        launch_fill(m->gtmp, m->n, 0.0, s);
        RAFEM_HIP(hipMemcpyAsync(m->bT, lambda_d, m->n * 8, hipMemcpyDeviceToDevice, s));
        launch_set_dirichlet(m->dir_ids, m->gtmp, m->nD, m->bT, s);
        if (!warm) launch_fill(m->adj_mu, m->n, 0.0, s);
        RAFEM_HIP(hipGetLastError());
        solve_any(m, o, step_matrix(m, m->valsT, m->valsT32), step_samples(m), m->dinvT,
                  m->dinvT32, m->bT, m->adj_mu, &inf.T, s, kSolveAdjointBioheat);
        if (inf.T.status != RAFEM_OK) {
            set_error("adjoint bioheat solve failed");
            return inf.T.status;
        }
        launch_vjp_params(npe, aff, m->E, m->conn, m->xyz, m->adj_mu, T_d, phys->T_a, grad_k_d,
                          grad_perf_d, s);
        const double* dsig = nullptr;
        if (phys->coupled) {
            launch_scatter_dirichlet(m->dir_ids, dir_V_d, m->nD, m->gV, s);
            assemble_potential(m, phys, sigma0_e_d, T_prev_d, s);
            launch_fill(m->rhs, m->n, 0.0, s);
            for (int c = 0; c < m->n_colours; ++c) {
                const int off = m->colour_off[c], cnt = m->colour_off[c + 1] - off;
                launch_vjp_joule_colour(npe, aff, m->colour_elems + off, cnt, m->conn, m->xyz, V_d,
                                        m->adj_mu, m->sigma, m->rhs, m->adj_sbar, s);
            }
            launch_set_dirichlet(m->dir_ids, m->gtmp, m->nD, m->rhs, s);
            if (!warm_nu) launch_fill(m->adj_nu, m->n, 0.0, s);
            RAFEM_HIP(hipGetLastError());
            solve_any(m, o, step_matrix(m, m->valsV, m->valsV32), step_samples(m), m->dinvV,
                      m->dinvV32, m->rhs, m->adj_nu, &inf.V, s, kSolveAdjointPotential);
            if (inf.V.status != RAFEM_OK) {
                set_error("adjoint potential solve failed");
                return inf.V.status;
            }
            launch_vjp_sigma(npe, aff, m->E, m->conn, m->xyz, m->adj_nu, V_d, m->adj_sbar,
                             sigma0_e_d, phys->alpha_sigma, m->adj_dsig, s);
            dsig = m->adj_dsig;
        }
        launch_fill(lambda_d, m->n, 0.0, s);
        for (int c = 0; c < m->n_colours; ++c) {
            const int off = m->colour_off[c], cnt = m->colour_off[c + 1] - off;
            launch_vjp_lambda_colour(npe, aff, m->colour_elems + off, cnt, m->conn, m->xyz,
                                     m->adj_mu, dsig, phys->rho_c / phys->dt, lambda_d, s);
        }
        RAFEM_HIP(hipGetLastError());
        m->adj_kept = phys->extrapolate != 0;
        m->adj_kept_nu = m->adj_kept && phys->coupled;
        return RAFEM_OK;
    });
}

rafem_status rafem_lesion_loss(rafem_mesh m, int64_t n_loss, const int32_t* ids_d,
                               const double* target_d, const double* T_d, double scale,
                               double* loss_d, double* grad_d, void* stream) {
    return guard([&]() -> rafem_status {
        check_device(m);
        require(n_loss >= 0 && n_loss <= m->n, "n_loss out of range");
        require(T_d && loss_d && (n_loss == 0 || (ids_d && target_d)), "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        double* grad = grad_d ? grad_d : m->gtmp;
        launch_fill(grad, m->n, 0.0, s);
        launch_loss(n_loss, ids_d, target_d, T_d, scale, grad, m->partials, loss_d, s);
        RAFEM_HIP(hipGetLastError());
        return RAFEM_OK;
    });
}

}  // extern "C"
