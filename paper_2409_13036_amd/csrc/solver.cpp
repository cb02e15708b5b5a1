// Host drivers of the Jacobi-PCG solves: FP64 PCG and FP32-inner / FP64-refined PCG.
//
// All arithmetic runs in the kernels; the host only enqueues chunks of
// iterations and polls the device-resident solver state between chunks.  The
// chunk length is predicted from the observed convergence rate so that few
// iterations are enqueued past convergence (those exit at once on the device
// flag) and the host synchronises only a handful of times per solve.
#include <algorithm>
#include <cmath>

#include "solver.hpp"

namespace rafem {

namespace {

void poll(rafem_mesh m, hipStream_t s) {
    RAFEM_HIP(hipMemcpyAsync(m->st_host, m->st, 3 * sizeof(PcgState), hipMemcpyDeviceToHost, s));
    RAFEM_HIP(hipStreamSynchronize(s));
}

// Iterations still needed to take rr down to tol2, from the rate seen between two polls.
int predict_chunk(double rr_prev, int it_prev, double rr, int it, double tol2, int fallback) {
    if (it > it_prev && rr_prev > 0.0 && rr > 0.0 && rr < rr_prev && tol2 > 0.0) {
        const double rate = std::log(rr / rr_prev) / double(it - it_prev);  // < 0
        const double need = std::log(tol2 / rr) / rate;
        if (std::isfinite(need)) return std::max(1, std::min(1024, (int)std::ceil(need * 1.02) + 1));
    }
    return fallback;
}

int first_chunk(const SolveOpts& o, int hint) {
    if (o.poll_every > 0) return o.poll_every;
    if (hint > 0) return std::max(1, (int)(hint * 0.95));
    return 16;
}

void check_launch() { RAFEM_HIP(hipGetLastError()); }

// Event pairs around the first launches of a chunk (measurement mode only).
struct ChunkTimer {
    rafem_mesh m;
    int rec = 0;
    int kind;
    ChunkTimer(rafem_mesh mm, int k, int which) : m(mm), kind(which) {
        rec = m->prof_on ? std::min(k, kProfCap) : 0;
    }
    void before(int j, hipStream_t s) {
        if (j < rec) RAFEM_HIP(hipEventRecord(m->prof_ev[2 * j], s));
    }
    void after(int j, hipStream_t s) {
        if (j < rec) RAFEM_HIP(hipEventRecord(m->prof_ev[2 * j + 1], s));
    }
    // after the stream has been synchronised: launches j with it_before + j < iters ran
    void collect(int it_before, int iters) {
        for (int j = 0; j < rec; ++j) {
            if (it_before + j >= iters) break;
            float ms = 0.f;
            RAFEM_HIP(hipEventElapsedTime(&ms, m->prof_ev[2 * j], m->prof_ev[2 * j + 1]));
            m->prof_sum_us[kind] += 1000.0 * ms;
            m->prof_cnt[kind] += 1;
        }
    }
};

}  // namespace

SolveOpts resolve_opts(const rafem_solve_opts* o, double default_tol) {
    SolveOpts r;
    r.tol = default_tol;
    if (o) {
        if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) throw Error{RAFEM_E_ARG, "opts.tol must be finite and >= 0"};
        if (o->precision != RAFEM_FP64 && o->precision != RAFEM_MIXED)
            throw Error{RAFEM_E_ARG, "opts.precision must be RAFEM_FP64 or RAFEM_MIXED"};
        if (o->inner_tol < 0.0 || o->inner_tol >= 1.0) throw Error{RAFEM_E_ARG, "opts.inner_tol must be in [0, 1)"};
        r.tol = o->tol;
        r.maxit = o->maxit > 0 ? o->maxit : 20000;
        r.precision = o->precision;
        r.inner_tol = o->inner_tol > 0.0 ? o->inner_tol : 1e-4;
        r.max_outer = o->max_outer > 0 ? o->max_outer : 30;
        r.poll_every = o->poll_every;
    }
    return r;
}

rafem_status pcg64(rafem_mesh m, const Mat& A, const double* dinv_in, const double* b, double* x,
                   const SolveOpts& o, rafem_solve_info* info, hipStream_t s, int hint,
                   int* iters_out) {
    PcgState* st = m->st;
    PcgState* chk = m->st + 2;
    const SpmvConfig& cfg = m->spmv;
    const int n = A.n;
    launch_state_init(st, o.tol, o.maxit, s);
    const double* dinv = dinv_in;
    if (!dinv) {
        if (A.sell) throw Error{RAFEM_E_STATE, "slab-layout solve without a Jacobi inverse"};
        launch_diag_inv(A, m->dinv, nullptr, st, s);
        dinv = m->dinv;
    }
    launch_pcg_start(A, cfg, b, x, dinv, m->r, m->p, m->partials, st, s);
    check_launch();

    int launched = 0;
    int chunk = first_chunk(o, hint);
    double rr_prev = -1.0;
    int it_prev = 0;
    PcgState& h = m->st_host[0];
    int it_before = 0;
    while (true) {
        const int k = std::min(chunk, o.maxit - launched);
        ChunkTimer timer(m, k, 0);
        for (int j = 0; j < k; ++j) {
            const int it = launched + j;
            timer.before(j, s);
            const int nb1 = launch_spmv_dot64(A, cfg, m->p, m->q, m->part_pq, st, s);
            timer.after(j, s);
            const int nb2 = launch_update64(n, x, m->r, m->p, m->q, dinv, m->part_pq, nb1,
                                            m->part_rz, it, st, s);
            launch_pupdate64(n, m->p, m->r, dinv, m->part_rz, nb2, it, st, s);
        }
        check_launch();
        launched += k;
        poll(m, s);
        timer.collect(it_before, h.iters);
        it_before = h.iters;
        if (h.done || launched >= o.maxit) break;
        if (rr_prev < 0.0) {
            rr_prev = h.rr_first;
            it_prev = 0;
        }
        const int fallback = o.poll_every > 0 ? o.poll_every : std::max(8, chunk);
        chunk = o.poll_every > 0 ? o.poll_every
                                 : predict_chunk(rr_prev, it_prev, h.rr, h.iters, h.tol2, fallback);
        rr_prev = h.rr;
        it_prev = h.iters;
    }
    const int status = h.status;
    const int iters = h.iters;
    const double bb = h.bb;
    const double relres = bb > 0.0 ? std::sqrt(h.rr / bb) : std::sqrt(h.rr);
    // True residual of the returned iterate.
    launch_state_init(chk, 0.0, 0, s);
    launch_residual64(A, cfg, b, x, m->r, m->partials, chk, 0, s);
    check_launch();
    poll(m, s);
    const PcgState& c = m->st_host[2];
    if (info) {
        info->status = status;
        info->iters = iters;
        info->outer = 0;
        info->launched = launched;
        info->relres = relres;
        info->relres_true = c.bb > 0.0 ? std::sqrt(c.rr / c.bb) : std::sqrt(c.rr);
    }
    if (iters_out) *iters_out = iters;
    return status;
}

rafem_status pcg_mixed(rafem_mesh m, const Mat& A, const double* dinv_in,
                       const float* dinv32_in, const double* b, double* x, const SolveOpts& o,
                       rafem_solve_info* info, hipStream_t s, int hint, int* iters_out) {
    PcgState* inner = m->st;
    PcgState* outer = m->st + 1;
    const SpmvConfig& cfg = m->spmv;
    const int n = A.n;
    launch_state_init(outer, o.tol, o.max_outer, s);
    const double* dinv = dinv_in;
    const float* dinv32 = dinv32_in;
    if (!dinv || !dinv32) {
        if (A.sell) throw Error{RAFEM_E_STATE, "slab-layout solve without a Jacobi inverse"};
        launch_diag_inv(A, m->dinv, m->dinv32, outer, s);
        dinv = m->dinv;
        dinv32 = m->dinv32;
    }
    int total_inner = 0, launched_total = 0, outer_steps = 0;
    int chunk0 = first_chunk(o, hint);
    double prev_outer_rr = -1.0;
    int stagnant = 0;
    bool fell_back = false;
    PcgState& hi = m->st_host[0];
    PcgState& ho = m->st_host[1];
    while (true) {
        launch_residual64(A, cfg, b, x, m->r64, m->partials, outer, 1, s);
        launch_inner_start(n, m->r64, outer, m->r32, m->d32, m->p32, dinv32, o.inner_tol,
                           o.maxit, m->partials, inner, s);
        check_launch();
        poll(m, s);  // outer convergence is decided by the residual just computed
        if (ho.done) break;
        int launched = 0;
        int chunk = chunk0;
        double rr_prev = -1.0;
        int it_prev = 0;
        int it_before = 0;
        while (true) {
            const int k = std::min(chunk, o.maxit - launched);
            ChunkTimer timer(m, k, 1);
            for (int j = 0; j < k; ++j) {
                const int it = launched + j;
                timer.before(j, s);
                const int nb1 = launch_spmv_dot32(A, cfg, m->p32, m->q32, m->part_pq, inner, s);
                timer.after(j, s);
                const int nb2 = launch_update32(n, m->d32, m->r32, m->p32, m->q32, dinv32,
                                                m->part_pq, nb1, m->part_rz, it, inner, s);
                launch_pupdate32(n, m->p32, m->r32, dinv32, m->part_rz, nb2, it, inner, s);
            }
            check_launch();
            launched += k;
            poll(m, s);
            timer.collect(it_before, hi.iters);
            it_before = hi.iters;
            if (hi.done || launched >= o.maxit) break;
            if (rr_prev < 0.0) {
                rr_prev = hi.rr_first;
                it_prev = 0;
            }
            chunk = o.poll_every > 0 ? o.poll_every
                                     : predict_chunk(rr_prev, it_prev, hi.rr, hi.iters, hi.tol2,
                                                     std::max(8, chunk));
            rr_prev = hi.rr;
            it_prev = hi.iters;
        }
        total_inner += hi.iters;
        launched_total += launched;
        outer_steps += 1;
        // next inner solve: the same number of iterations is a good first guess
        if (o.poll_every <= 0 && hi.iters > 0) chunk0 = std::max(1, (int)(hi.iters * 0.95));
        launch_refine_update(n, x, m->d32, outer, s);
        check_launch();
        // stagnation: the FP64 residual must at least halve per refinement
        if (prev_outer_rr > 0.0 && ho.rr > 0.25 * prev_outer_rr) stagnant += 1;
        else stagnant = 0;
        prev_outer_rr = ho.rr;
        if (stagnant >= 2) {
            fell_back = true;
            break;
        }
    }
    if (fell_back) {
        rafem_solve_info sub{};
        SolveOpts o64 = o;
        o64.precision = RAFEM_FP64;
        int it64 = 0;
        rafem_status st = pcg64(m, A, dinv, b, x, o64, &sub, s, 0, &it64);
        if (info) {
            *info = sub;
            info->iters = total_inner + sub.iters;
            info->outer = -outer_steps;  // negative: refinement stagnated, FP64 PCG finished
            info->launched = launched_total + sub.launched;
        }
        if (iters_out) *iters_out = total_inner + it64;
        return st;
    }
    const int status = ho.status;
    if (info) {
        info->status = status;
        info->iters = total_inner;
        info->outer = outer_steps;
        info->launched = launched_total;
        info->relres = ho.bb > 0.0 ? std::sqrt(ho.rr / ho.bb) : std::sqrt(ho.rr);
        info->relres_true = info->relres;  // the refinement residual is the true FP64 residual
    }
    if (iters_out) *iters_out = total_inner;
    return status;
}

}  // namespace rafem
