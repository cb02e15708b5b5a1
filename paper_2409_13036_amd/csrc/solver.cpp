// Host drivers of the Jacobi-PCG solves: FP64 PCG and FP32-inner / FP64-refined PCG,
// for one system or a batch of independent systems (one state per sample).
//
// All arithmetic runs in the kernels; the host only enqueues chunks of iterations and
// polls the device-resident solver states between chunks.  The chunk length is
// predicted from the observed convergence rate of the slowest sample, so few iterations
// are enqueued past convergence (those exit at once on the device flag) and the host
// synchronises only a handful of times per solve.  Optionally a chunk is captured once
// as a HIP graph (its iteration index comes from device memory) and replayed.
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "solver.hpp"

namespace rafem {

namespace {

void check_launch() { RAFEM_HIP(hipGetLastError()); }

void poll(rafem_mesh m, hipStream_t s) {
    RAFEM_HIP(hipMemcpyAsync(m->st_host, m->st, 3 * m->S * sizeof(PcgState), hipMemcpyDeviceToHost,
                             s));
    RAFEM_HIP(hipStreamSynchronize(s));
}

// Iterations still needed to take rr down to tol2, from the rate seen between two polls.
int predict_one(double rr_prev, int it_prev, double rr, int it, double tol2, int fallback) {
    if (it > it_prev && rr_prev > 0.0 && rr > 0.0 && rr < rr_prev && tol2 > 0.0) {
        const double rate = std::log(rr / rr_prev) / double(it - it_prev);  // < 0
        const double need = std::log(tol2 / rr) / rate;
        // a launch past convergence costs a few microseconds, a poll tens: overshoot a little
        if (std::isfinite(need)) return std::max(1, std::min(1024, (int)std::ceil(need * 1.03) + 2));
    }
    return fallback;
}

int first_chunk(const SolveOpts& o, int hint) {
    if (o.poll_every > 0) return o.poll_every;
    if (hint > 0) return hint;
    return 16;
}

int hint_at(const std::vector<int>* hints, size_t k) {
    return hints && k < hints->size() ? (*hints)[k] : 0;
}

// Tracks the convergence of every unfinished sample between polls.
struct Predictor {
    std::vector<double> rr_prev;
    std::vector<int> it_prev;
    explicit Predictor(int S) : rr_prev(S, -1.0), it_prev(S, 0) {}
    int next(const PcgState* h, int S, int fallback) {
        int need = 0;
        bool any = false;
        for (int s = 0; s < S; ++s) {
            if (h[s].done) continue;
            any = true;
            if (rr_prev[s] < 0.0) {
                rr_prev[s] = h[s].rr_first;
                it_prev[s] = 0;
            }
            need = std::max(need, predict_one(rr_prev[s], it_prev[s], h[s].rr, h[s].iters,
                                              h[s].tol2, fallback));
            rr_prev[s] = h[s].rr;
            it_prev[s] = h[s].iters;
        }
        return any ? std::max(1, need) : fallback;
    }
};

bool all_done(const PcgState* h, int S) {
    for (int s = 0; s < S; ++s)
        if (!h[s].done) return false;
    return true;
}

int max_iters(const PcgState* h, int S) {
    int it = 0;
    for (int s = 0; s < S; ++s) it = std::max(it, h[s].iters);
    return it;
}

int worst_status(const PcgState* h, int S) {
    int status = RAFEM_OK;
    for (int s = 0; s < S; ++s)
        if (h[s].status != RAFEM_OK) status = std::max(status, h[s].status);
    return status;
}

// Event pairs stamped at the start and end of the SpMV kernels of a chunk (measurement
// mode, no graphs).
struct ChunkTimer {
    rafem_mesh m;
    int rec = 0;
    int kind;
    ChunkTimer(rafem_mesh mm, int k, int which) : m(mm), kind(which) {
        rec = m->prof_on ? std::min(k, kProfCap) : 0;
    }
    hipEvent_t start(int j) const { return j < rec ? m->prof_ev[2 * j] : nullptr; }
    hipEvent_t stop(int j) const { return j < rec ? m->prof_ev[2 * j + 1] : nullptr; }
    // after the stream has been synchronised: launch j ran iff it_before + j < iters
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

// One FP64 PCG iteration (three kernels) at offset j of a chunk.
struct Iter64 {
    rafem_mesh m;
    const Mat* A;
    const SpmvConfig* cfg;
    const double* dinv;
    double* x;
    PcgState* st;
    Samples smp;
    int* itb;
    void operator()(int j, hipStream_t s, ChunkTimer* t) const {
        const int n = A->n;
        const GridInfo g1 = launch_spmv_dot64(*A, *cfg, m->p, m->q, m->part_pq, st, smp, s,
                                              t ? t->start(j) : nullptr, t ? t->stop(j) : nullptr);
        const int nb2 = launch_update64(n, x, m->r, m->p, m->q, dinv, m->part_pq, g1, m->part_rz,
                                        itb, j, st, smp, m->part_sum, s);
        launch_pupdate64(n, m->p, m->r, m->part_rz, nb2, itb, j, st, smp, m->part_sum, s);
    }
};

// One FP32 inner iteration.
struct Iter32 {
    rafem_mesh m;
    const Mat* A;
    const SpmvConfig* cfg;
    const float* dinv32;
    PcgState* st;
    Samples smp;
    int* itb;
    void operator()(int j, hipStream_t s, ChunkTimer* t) const {
        const int n = A->n;
        const GridInfo g1 = launch_spmv_dot32(*A, *cfg, m->p32, m->q32, m->part_pq, st, smp, s,
                                              t ? t->start(j) : nullptr, t ? t->stop(j) : nullptr);
        const int nb2 = launch_update32(n, m->d32, m->r32, m->p32, m->q32, dinv32, m->part_pq, g1,
                                        m->part_rz, itb, j, st, smp, m->part_sum, s);
        launch_pupdate32(n, m->p32, m->r32, m->part_rz, nb2, itb, j, st, smp, m->part_sum, s);
    }
};

constexpr int kGraphLen = 8;     // iterations per captured chunk
constexpr size_t kMaxGraphs = 16;  // graphs kept per mesh (callers that keep changing their
                                   // buffers would otherwise grow the cache without bound)

// The graph of kGraphLen iterations for this set of buffers, captured on first use.
template <typename IT>
hipGraphExec_t chunk_graph(rafem_mesh m, int kind, const void* k0, const void* k1,
                           const void* k2, const void* k3, const IT& iter, int* itb) {
    for (auto& g : m->graphs)
        if (g.kind == kind && g.key[0] == k0 && g.key[1] == k1 && g.key[2] == k2 &&
            g.key[3] == k3 && g.len == kGraphLen)
            return g.exec;
    if (m->graphs.size() >= kMaxGraphs) {  // drop the oldest
        (void)hipGraphExecDestroy(m->graphs.front().exec);
        m->graphs.erase(m->graphs.begin());
    }
    if (!m->gstream) RAFEM_HIP(hipStreamCreateWithFlags(&m->gstream, hipStreamNonBlocking));
    RAFEM_HIP(hipStreamBeginCapture(m->gstream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < kGraphLen; ++j) iter(j, m->gstream, nullptr);
    launch_advance(itb, kGraphLen, m->gstream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(m->gstream, &graph);
    if (e != hipSuccess)
        throw Error{RAFEM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e)};
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess)
        throw Error{RAFEM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e2)};
    m->graphs.push_back({kind, {k0, k1, k2, k3}, kGraphLen, exec});
    return exec;
}

// Enqueue k iterations: whole chunks as replays of the captured graph (one host call per
// kGraphLen iterations), the rest as stream launches.  Both advance the same device
// iteration counter, so the mix runs exactly the iterations of stream launches alone.
template <typename IT>
int enqueue(int k, const IT& iter, hipGraphExec_t graph, int* itb, ChunkTimer* t, hipStream_t s) {
    int done = 0;
    if (graph) {
        for (; done + kGraphLen <= k; done += kGraphLen) RAFEM_HIP(hipGraphLaunch(graph, s));
        if (done == k) return k;
    }
    const int rest = k - done;
    for (int j = 0; j < rest; ++j) iter(j, s, t);
    launch_advance(itb, rest, s);
    return k;
}

void fill_info(rafem_solve_info* info, const PcgState* h, const PcgState* chk, int S, int launched,
               int outer) {
    if (!info) return;
    double relres = 0.0, relres_true = 0.0;
    for (int s = 0; s < S; ++s) {
        const double bb = h[s].bb;
        relres = std::max(relres, bb > 0.0 ? std::sqrt(h[s].rr / bb) : std::sqrt(h[s].rr));
        if (chk) {
            const double cb = chk[s].bb;
            relres_true = std::max(relres_true,
                                   cb > 0.0 ? std::sqrt(chk[s].rr / cb) : std::sqrt(chk[s].rr));
        }
    }
    info->status = worst_status(h, S);
    info->iters = max_iters(h, S);
    info->outer = outer;
    info->launched = launched;
    info->relres = relres;
    info->relres_true = chk ? relres_true : relres;
}

}  // namespace

SolveOpts resolve_opts(const rafem_solve_opts* o, double default_tol) {
    SolveOpts r;
    r.tol = default_tol;
    if (o) {
        if (!(o->tol >= 0.0) || !std::isfinite(o->tol))
            throw Error{RAFEM_E_ARG, "opts.tol must be finite and >= 0"};
        if (o->precision != RAFEM_FP64 && o->precision != RAFEM_MIXED)
            throw Error{RAFEM_E_ARG, "opts.precision must be RAFEM_FP64 or RAFEM_MIXED"};
        if (o->inner_tol < 0.0 || o->inner_tol >= 1.0)
            throw Error{RAFEM_E_ARG, "opts.inner_tol must be in [0, 1)"};
        r.tol = o->tol;
        r.maxit = o->maxit > 0 ? o->maxit : 20000;
        r.precision = o->precision;
        r.inner_tol = o->inner_tol > 0.0 ? o->inner_tol : 3e-5;
        r.max_outer = o->max_outer > 0 ? o->max_outer : 30;
        r.poll_every = o->poll_every;
        if (o->restart_inner != 0 && o->restart_inner != 1)
            throw Error{RAFEM_E_ARG, "opts.restart_inner must be 0 or 1"};
        r.restart_inner = o->restart_inner;
    }
    return r;
}

rafem_status pcg64(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv_in,
                   const double* b, double* x, const SolveOpts& o, rafem_solve_info* info,
                   hipStream_t s, std::vector<int>* hints) {
    const int S = smp.S;
    PcgState* st = m->st;
    PcgState* chk = m->st + 2 * S;
    const SpmvConfig& cfg = m->spmv;
    int* itb = m->itb;
    launch_state_init(st, S, o.tol, o.maxit, itb, s);
    const double* dinv = dinv_in;
    if (!dinv) {
        if (A.sell || S != 1) throw Error{RAFEM_E_STATE, "slab-layout solve without a Jacobi inverse"};
        launch_diag_inv(A, m->dinv, nullptr, st, s);
        dinv = m->dinv;
    }
    launch_pcg_start(A, cfg, b, x, dinv, m->r, m->p, m->partials, st, smp, s);
    check_launch();

    const Iter64 iter{m, &A, &cfg, dinv, x, st, smp, itb};
    hipGraphExec_t graph = nullptr;
    if ((m->use_graphs || (m->graphs_small && hints)) && !m->prof_on)
        graph = chunk_graph(m, 0, A.v, x, dinv, A.sell ? (const void*)A.sptr : (const void*)A.rp,
                            iter, itb);
    int launched = 0;
    int chunk = first_chunk(o, hint_at(hints, 0));
    Predictor pred(S);
    const PcgState* h = m->st_host;
    while (true) {
        const int k = std::min(chunk, o.maxit - launched);
        ChunkTimer timer(m, graph ? 0 : k, 0);
        const int it_before = launched;
        launched += enqueue(k, iter, graph, itb, &timer, s);
        check_launch();
        poll(m, s);
        timer.collect(it_before, max_iters(h, S));
        if (all_done(h, S) || launched >= o.maxit) break;
        const int fallback = o.poll_every > 0 ? o.poll_every : std::max(8, chunk);
        chunk = o.poll_every > 0 ? o.poll_every : pred.next(h, S, fallback);
    }
    const int iters = max_iters(h, S);
    // true residual of the returned iterates
    launch_state_init(chk, S, 0.0, 0, nullptr, s);
    launch_residual64(A, cfg, b, x, m->r, m->partials, chk, smp, 0, s);
    check_launch();
    poll(m, s);
    fill_info(info, h, h + 2 * S, S, launched, 0);
    if (hints) hints->assign(1, iters);
    return worst_status(h, S);
}

rafem_status pcg_mixed(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv_in,
                       const float* dinv32_in, const double* b, double* x, const SolveOpts& o,
                       rafem_solve_info* info, hipStream_t s, std::vector<int>* hints) {
    const int S = smp.S;
    PcgState* inner = m->st;
    PcgState* outer = m->st + S;
    const int n = A.n;
    int* itb = m->itb + 1;
    launch_state_init(outer, S, o.tol, o.max_outer, nullptr, s);
    const double* dinv = dinv_in;
    const float* dinv32 = dinv32_in;
    if (!dinv || !dinv32) {
        if (A.sell || S != 1) throw Error{RAFEM_E_STATE, "slab-layout solve without a Jacobi inverse"};
        launch_diag_inv(A, m->dinv, m->dinv32, outer, s);
        dinv = m->dinv;
        dinv32 = m->dinv32;
    }
    const Iter32 iter{m, &A, &m->spmv32, dinv32, inner, smp, itb};
    hipGraphExec_t graph = nullptr;
    if ((m->use_graphs || (m->graphs_small && hints)) && !m->prof_on)
        graph = chunk_graph(m, 1, A.v32, dinv32, A.sell ? (const void*)A.sptr : (const void*)A.rp,
                            nullptr, iter, itb);
    int total_inner = 0, launched_total = 0, outer_steps = 0;
    m->mixed_iters.assign(S, 0);
    m->mixed_fell.assign(S, 0);
    std::vector<int> counts;  // iterations of each inner solve
    std::vector<double> prev_rr(S, -1.0);
    std::vector<int> stagnant(S, 0);
    bool fell_back = false;
    const PcgState* hi = m->st_host;
    PcgState* ho = m->st_host + S;
    while (true) {
        launch_residual64(A, m->spmv, b, x, m->r64, m->partials, outer, smp, 1, s);
        // the first refinement starts the inner recurrence, later ones continue it from the
        // refined residual (unless plain restarted refinement is asked for)
        const int cont = (outer_steps > 0 && !o.restart_inner) ? 1 : 0;
        launch_inner_start(n, m->r64, outer, m->r32, m->d32, m->p32, dinv32, o.inner_tol, o.maxit,
                           m->partials, inner, smp, cont, s);
        launch_state_init(nullptr, 0, 0.0, 0, itb, s);  // inner iteration counter = 0
        check_launch();
        poll(m, s);  // outer convergence is decided by the residuals just computed
        if (all_done(ho, S)) break;
        int launched = 0;
        // first chunk: the same inner solve of the previous solve, else 90% of this one's last
        int guess = hint_at(hints, counts.size());
        if (guess <= 0 && !counts.empty()) guess = std::max(1, (int)(counts.back() * 0.9));
        int chunk = first_chunk(o, guess);
        Predictor pred(S);
        while (true) {
            const int k = std::min(chunk, o.maxit - launched);
            ChunkTimer timer(m, graph ? 0 : k, 1);
            const int it_before = launched;
            launched += enqueue(k, iter, graph, itb, &timer, s);
            check_launch();
            poll(m, s);
            timer.collect(it_before, max_iters(hi, S));
            if (all_done(hi, S) || launched >= o.maxit) break;
            chunk = o.poll_every > 0 ? o.poll_every : pred.next(hi, S, std::max(8, chunk));
        }
        const int it_in = max_iters(hi, S);
        total_inner += it_in;
        counts.push_back(it_in);
        for (int q = 0; q < S; ++q) m->mixed_iters[q] += hi[q].iters;
        launched_total += launched;
        outer_steps += 1;
        launch_refine_update(n, x, m->d32, outer, smp, s);
        check_launch();
        // Stagnation: each unfinished sample's FP64 residual must fall 4x per refinement.  A
        // sample that fails twice is frozen (its refinement state is marked done, after the
        // update just enqueued) and FP64 PCG finishes it once every other sample is through,
        // so a sample's iterates never depend on the other samples of a batch.
        bool frozen = false;
        for (int q = 0; q < S; ++q) {
            if (ho[q].done) continue;
            if (prev_rr[q] > 0.0 && ho[q].rr > 0.25 * prev_rr[q]) stagnant[q] += 1;
            else stagnant[q] = 0;
            prev_rr[q] = ho[q].rr;
            if (stagnant[q] >= 2) {
                ho[q].done = 1;
                m->mixed_fell[q] = 1;
                frozen = true;
            }
        }
        if (frozen) {
            // the host copy of the refinement states is current: only the inner states have
            // changed on the device since the last poll
            RAFEM_HIP(hipMemcpyAsync(outer, ho, S * sizeof(PcgState), hipMemcpyHostToDevice, s));
            fell_back = true;
        }
    }
    if (fell_back) {
        // samples that converged under refinement exit FP64 PCG at once (its start computes
        // the same residual), so only the frozen ones move
        rafem_solve_info sub{};
        SolveOpts o64 = o;
        o64.precision = RAFEM_FP64;
        const rafem_status st = pcg64(m, A, smp, dinv, b, x, o64, &sub, s, nullptr);
        for (int q = 0; q < S; ++q) m->mixed_iters[q] += m->st_host[q].iters;
        if (info) {
            *info = sub;
            info->iters = total_inner + sub.iters;
            info->outer = -outer_steps;  // negative: refinement stagnated, FP64 PCG finished
            info->launched = launched_total + sub.launched;
        }
        if (hints) *hints = counts;
        return st;
    }
    // the refinement residual is the true FP64 residual of the returned iterate
    fill_info(info, ho, nullptr, S, launched_total, outer_steps);
    if (info) info->iters = total_inner;
    if (hints) *hints = counts;
    return worst_status(ho, S);
}

void solve_enqueue(rafem_mesh m, const Mat& A, const Samples& smp, const double* b, double* x,
                   const SolveOpts& o, int iterations, int refinements,
                   rafem_device_info* info_d, hipStream_t s) {
    // the sequence of pcg64 / pcg_mixed with the host polls taken out: kernels of a solve,
    // inner solve or refinement that has finished exit at their first instruction
    launch_info_begin(info_d, s);
    PcgState* chk = m->st + 2;
    if (o.precision != RAFEM_MIXED) {
        PcgState* st = m->st;
        int* itb = m->itb;
        launch_state_init(st, 1, o.tol, iterations, itb, s);
        launch_diag_inv(A, m->dinv, nullptr, st, s);
        launch_pcg_start(A, m->spmv, b, x, m->dinv, m->r, m->p, m->partials, st, smp, s);
        const Iter64 iter{m, &A, &m->spmv, m->dinv, x, st, smp, itb};
        enqueue(iterations, iter, nullptr, itb, nullptr, s);
        launch_state_init(chk, 1, 0.0, 0, nullptr, s);
        launch_residual64(A, m->spmv, b, x, m->r, m->partials, chk, smp, 0, s);
        launch_info_finish(st, chk, 0, info_d, s);
        check_launch();
        return;
    }
    PcgState* inner = m->st;
    PcgState* outer = m->st + 1;
    int* itb = m->itb + 1;
    const int n = A.n;
    launch_state_init(outer, 1, o.tol, refinements, nullptr, s);
    launch_diag_inv(A, m->dinv, m->dinv32, outer, s);
    const Iter32 iter{m, &A, &m->spmv32, m->dinv32, inner, smp, itb};
    for (int j = 0;; ++j) {
        launch_residual64(A, m->spmv, b, x, m->r64, m->partials, outer, smp, 1, s);
        if (j == refinements) break;  // the residual check of the last refinement
        const int cont = (j > 0 && !o.restart_inner) ? 1 : 0;
        launch_inner_start(n, m->r64, outer, m->r32, m->d32, m->p32, m->dinv32, o.inner_tol,
                           o.maxit, m->partials, inner, smp, cont, s);
        launch_state_init(nullptr, 0, 0.0, 0, itb, s);
        enqueue(iterations, iter, nullptr, itb, nullptr, s);
        launch_refine_update(n, x, m->d32, outer, smp, s);
        launch_info_add_inner(inner, info_d, s);
    }
    launch_info_finish(outer, outer, 1, info_d, s);
    check_launch();
}

bool dd_ready(rafem_mesh m, const SolveOpts& o, const std::vector<int>* hints) {
    if (!m->dd_on || m->prof_on || !hints || hints->empty() || o.poll_every > 0) return false;
    const int rounds = o.precision == RAFEM_MIXED ? (int)hints->size() + 1 : 1;
    if (o.precision == RAFEM_MIXED && rounds > std::min(kDdMaxRounds, o.max_outer + 1)) return false;
    return m->dd_used + rounds <= kDdSlots;
}

namespace {

int dd_budget(rafem_mesh m, int count, int maxit) {
    const int k = (int)std::ceil(count * m->dd_scale) + kDdSlack;
    return std::max(1, std::min(k, maxit));
}


void dd_log(rafem_mesh m, int slot, hipStream_t s) {
    const size_t n = 3 * (size_t)m->S;
    RAFEM_HIP(hipMemcpyAsync(m->dd_log + slot * n, m->st, n * sizeof(PcgState),
                             hipMemcpyDeviceToDevice, s));
}

}  // namespace

DdRecord dd_enqueue(rafem_mesh m, const Mat& A, const Samples& smp, const double* dinv,
                    const float* dinv32, const double* b, double* x, const SolveOpts& o,
                    const std::vector<int>& hints, hipStream_t s) {
    const int S = smp.S;
    DdRecord r;
    r.slot0 = m->dd_used;
    r.mixed = o.precision == RAFEM_MIXED;
    if (!r.mixed) {
        PcgState* st = m->st;
        PcgState* chk = m->st + 2 * S;
        int* itb = m->itb;
        launch_state_init(st, S, o.tol, o.maxit, itb, s);
        launch_pcg_start(A, m->spmv, b, x, dinv, m->r, m->p, m->partials, st, smp, s);
        const Iter64 iter{m, &A, &m->spmv, dinv, x, st, smp, itb};
        hipGraphExec_t graph = nullptr;
        if (m->use_graphs)
            graph = chunk_graph(m, 0, A.v, x, dinv, (const void*)A.sptr, iter, itb);
        const int k = dd_budget(m, hints[0], o.maxit);
        enqueue(k, iter, graph, itb, nullptr, s);
        launch_state_init(chk, S, 0.0, 0, nullptr, s);
        launch_residual64(A, m->spmv, b, x, m->r, m->partials, chk, smp, 0, s);
        dd_log(m, r.slot0, s);
        check_launch();
        r.rounds = 1;
        r.budget.push_back(k);
        m->dd_used += 1;
        return r;
    }
    PcgState* inner = m->st;
    PcgState* outer = m->st + S;
    const int n = A.n;
    int* itb = m->itb + 1;
    launch_state_init(outer, S, o.tol, o.max_outer, nullptr, s);
    const Iter32 iter{m, &A, &m->spmv32, dinv32, inner, smp, itb};
    hipGraphExec_t graph = nullptr;
    if (m->use_graphs)
        graph = chunk_graph(m, 1, A.v32, dinv32, (const void*)A.sptr, nullptr, iter, itb);
    const int rounds = (int)hints.size() + 1;
    for (int j = 0; j < rounds; ++j) {
        // the same sequence as pcg_mixed's loop; rounds past a sample's convergence leave its
        // x alone (every kernel skips a finished refinement)
        launch_residual64(A, m->spmv, b, x, m->r64, m->partials, outer, smp, 1, s);
        if (j == (int)hints.size()) {
            // the check round: the residual of the last refinement decides; a sample that
            // needs another refinement makes the step be redone
            dd_log(m, r.slot0 + j, s);
            r.budget.push_back(0);
            break;
        }
        const int cont = (j > 0 && !o.restart_inner) ? 1 : 0;
        launch_inner_start(n, m->r64, outer, m->r32, m->d32, m->p32, dinv32, o.inner_tol, o.maxit,
                           m->partials, inner, smp, cont, s);
        launch_state_init(nullptr, 0, 0.0, 0, itb, s);
        const int k = dd_budget(m, hints[j], o.maxit);
        enqueue(k, iter, graph, itb, nullptr, s);
        launch_refine_update(n, x, m->d32, outer, smp, s);
        dd_log(m, r.slot0 + j, s);
        r.budget.push_back(k);
    }
    check_launch();
    r.rounds = rounds;
    m->dd_used += rounds;
    return r;
}

bool dd_finish(rafem_mesh m, const DdRecord& r, const SolveOpts& o, rafem_solve_info* info,
               std::vector<int>* hints, const PcgState** h_out) {
    const int S = m->S;
    const size_t n = 3 * (size_t)S;
    const PcgState* log = m->dd_log_host + r.slot0 * n;
    if (!r.mixed) {
        const PcgState* h = log;
        for (int q = 0; q < S; ++q)
            if (!h[q].done || h[q].status != RAFEM_OK) return false;
        fill_info(info, h, h + 2 * S, S, r.budget[0], 0);
        if (hints) hints->assign(1, max_iters(h, S));
        *h_out = h;
        return true;
    }
    std::vector<double> prev_rr(S, -1.0);
    std::vector<int> stagnant(S, 0), per_sample(S, 0), counts;
    int total_inner = 0, launched = 0, outer_steps = 0;
    for (int j = 0; j < r.rounds; ++j) {
        const PcgState* in = log + j * n;
        const PcgState* out = in + S;
        bool ran = false;
        for (int q = 0; q < S; ++q) {
            if (out[q].done) continue;
            ran = true;
            if (!in[q].done) return false;  // the inner solve ran out of its budget
            // the host-driven solve's stagnation rule on the same residuals
            if (prev_rr[q] > 0.0 && out[q].rr > 0.25 * prev_rr[q]) stagnant[q] += 1;
            else stagnant[q] = 0;
            prev_rr[q] = out[q].rr;
            if (stagnant[q] >= 2) return false;
        }
        if (!ran) continue;
        const int it = max_iters(in, S);
        counts.push_back(it);
        total_inner += it;
        launched += r.budget[j];
        outer_steps += 1;
        for (int q = 0; q < S; ++q) per_sample[q] += in[q].iters;
    }
    const PcgState* last = log + (r.rounds - 1) * n;
    for (int q = 0; q < S; ++q)
        if (!last[S + q].done || last[S + q].status != RAFEM_OK) return false;
    m->mixed_iters = per_sample;
    m->mixed_fell.assign(S, 0);
    fill_info(info, last + S, nullptr, S, launched, outer_steps);
    if (info) info->iters = total_inner;
    if (hints) *hints = counts;
    *h_out = last;
    return true;
}

namespace {

// On-disk cache of the tuned SpMV configurations: one line per (device, layout) key,
// "<key> <slabs per block FP64> <slabs per block FP32> <streamed FP64> <streamed FP32>
// <resident slots FP64> <resident slots FP32> <launch bound FP64> <launch bound FP32>", in the
// file named by RAFEM_TUNE_CACHE, else
// $HOME/.cache/rafem/spmv_tune.txt.  Unreadable or unwritable files, and lines of another
// form, are ignored (the configurations are then timed).
std::string tune_cache_path() {
    if (const char* p = std::getenv("RAFEM_TUNE_CACHE")) return p;
    if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/rafem/spmv_tune.txt";
    return "";
}

std::string tune_key(rafem_mesh m) {
    hipDeviceProp_t prop{};
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) dev = prop.gcnArchName;
    for (char& c : dev)
        if (c == ' ') c = '_';
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s/n%lld/nnz%lld/slots%lld/slabs%d/shared%lld/S%d/i16%d",
                  dev.c_str(), (long long)m->n, (long long)m->nnz, (long long)m->sell_nnz,
                  m->nslabs, (long long)m->shared_slabs, m->S, m->sdel ? 1 : 0);
    return buf;
}

bool tune_lookup(const std::string& key, SpmvConfig& c64, SpmvConfig& c32) {
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    std::FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[640], k[512];
    int a = 0, b = 0, na = 0, nb = 0, ra = 0, rb = 0, ma = 0, mb = 0;
    bool found = false;
    auto bound_ok = [](int v) { return v == 1 || v == kSellMinBlocks; };
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line, "%511s %d %d %d %d %d %d %d %d", k, &a, &b, &na, &nb, &ra, &rb, &ma,
                        &mb) != 9)
            continue;
        if (key == k && (a == 8 || a == 16) && (b == 8 || b == 16) && (na == 0 || na == 1) &&
            (nb == 0 || nb == 1) && ra >= 0 && rb >= 0 && bound_ok(ma) &&
            bound_ok(mb)) {  // last entry wins
            c64.slabs_per_block = a;
            c32.slabs_per_block = b;
            c64.stream = na;
            c32.stream = nb;
            c64.resident = ra;
            c32.resident = rb;
            c64.min_blocks = ma;
            c32.min_blocks = mb;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const std::string& key, const SpmvConfig& c64, const SpmvConfig& c32) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // create the cache's folder and its parent if missing (errors ignored)
        const std::string dir = path.substr(0, slash);
        const size_t up = dir.rfind('/');
        if (up != std::string::npos && up > 0) (void)mkdir(dir.substr(0, up).c_str(), 0755);
        (void)mkdir(dir.c_str(), 0755);
    }
    std::FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", key.c_str(), c64.slabs_per_block,
                 c32.slabs_per_block, c64.stream, c32.stream, c64.resident, c32.resident,
                 c64.min_blocks, c32.min_blocks);
    std::fclose(f);
}

}  // namespace

void autotune_spmv(rafem_mesh m, const Mat& A, hipStream_t s) {
    // SELL kernel configuration: 2 or 4 slabs per wavefront (one or two groups of partial
    // sums per workgroup, so results do not depend on the choice), the kernel's launch bound
    // (the compiler's register budget, or one that keeps 6 workgroups per CU), and the matrix values
    // read with ordinary loads, or with nontemporal loads past a prefix of 0 or 96 MiB read
    // with ordinary ones (streaming pays when the values do not fit the Infinity Cache and
    // loses when they do, since the solve's products then re-read them from it; a prefix
    // can stay there while the rest streams past), chosen by timing the PCG SpMV (with its
    // fused dot product) on this mesh's matrix with a PCG iteration's vector traffic
    // between the products, as in the solve, for FP64 and FP32 values; or taken from the
    // on-disk cache of earlier timings of the same layout on the same kind of device.
    // Every candidate keeps workgroups inside one sample (kRowAlign is 16 slabs) and gives
    // the same bits.
    if (!A.sell) return;
    const std::string key = tune_key(m);
    if (tune_lookup(key, m->spmv, m->spmv32)) {
        m->tuned = true;
        m->tuned_from_cache = true;
        return;
    }
    const int S = m->S;
    Samples smp{S, m->row_off, m->row_tab};
    PcgState* chk = m->st + 2 * S;
    constexpr int kTuneReps = 5;
    constexpr double kTuneMargin = 0.98;
    hipEvent_t ev[2 * kTuneReps];
    for (hipEvent_t& e : ev) RAFEM_HIP(hipEventCreate(&e));
    launch_fill(m->p, m->n, 0.0, s);
    launch_fill32(m->p32, m->n, 0.0f, s);
    launch_state_init(chk, S, 0.0, 0, nullptr, s);
    for (int prec = 0; prec < 2; ++prec) {
        SpmvConfig& target = prec ? m->spmv32 : m->spmv;
        double best = 1e30;
        SpmvConfig best_c = target;
        // value-load candidates: ordinary; streamed past a prefix of 0 or 96 MiB (a prefix
        // that holds the whole matrix is the ordinary candidate again)
        const int64_t value_bytes = m->sell_nnz * (prec ? 4 : 8);
        std::vector<std::pair<int, int>> loads{{0, 0}};
        for (int64_t mib : {0, 96})
            if (mib * 1048576 < value_bytes)
                loads.push_back({1, (int)(mib * 1048576 / (prec ? 4 : 8))});
        for (int cand = 0; cand < 4 * (int)loads.size(); ++cand) {
            SpmvConfig c = target;
            c.slabs_per_block = 4 * (cand % 2 ? 4 : 2);
            c.min_blocks = (cand / 2) % 2 ? kSellMinBlocks : 1;
            c.stream = loads[cand / 4].first;
            c.resident = loads[cand / 4].second;
            auto run = [&](hipEvent_t a0, hipEvent_t a1) {
                if (prec) launch_spmv_dot32(A, c, m->p32, m->q32, m->part_pq, chk, smp, s, a0, a1);
                else launch_spmv_dot64(A, c, m->p, m->q, m->part_pq, chk, smp, s, a0, a1);
            };
            // between products, the vector traffic of a PCG iteration (four copies of a
            // vector: 8 words per row against the iteration's 10), which competes with the
            // matrix for the Infinity Cache as in the solve; only the products are timed
            auto sweep = [&]() {
                const size_t bytes = (size_t)m->n * (prec ? 4 : 8);
                void* v0 = prec ? (void*)m->r32 : (void*)m->r;
                void* v1 = prec ? (void*)m->q32 : (void*)m->q;
                for (int k = 0; k < 2; ++k) {
                    RAFEM_HIP(hipMemcpyAsync(v1, v0, bytes, hipMemcpyDeviceToDevice, s));
                    RAFEM_HIP(hipMemcpyAsync(v0, v1, bytes, hipMemcpyDeviceToDevice, s));
                }
            };
            for (int w = 0; w < 2; ++w) {
                run(nullptr, nullptr);
                sweep();
            }
            for (int r = 0; r < kTuneReps; ++r) {
                run(ev[2 * r], ev[2 * r + 1]);
                sweep();
            }
            RAFEM_HIP(hipEventSynchronize(ev[2 * kTuneReps - 1]));
            float ms = 0.f;
            for (int r = 0; r < kTuneReps; ++r) {
                float one = 0.f;
                RAFEM_HIP(hipEventElapsedTime(&one, ev[2 * r], ev[2 * r + 1]));
                ms += one;
            }
            // the capped launch bound must be 2% faster to be taken, so that timing noise
            // between kernels of equal occupancy (the FP32 ones hold 7 wavefronts per SIMD
            // either way) keeps the compiler's register budget
            const double eff = c.min_blocks == 1 ? ms : ms / kTuneMargin;
            if (eff < best) {
                best = eff;
                best_c = c;
            }
        }
        target = best_c;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    RAFEM_HIP(hipGetLastError());
    m->tuned = true;
    tune_store(key, m->spmv, m->spmv32);
}

}  // namespace rafem
