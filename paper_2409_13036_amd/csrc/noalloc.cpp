// Allocation-free variant of rafem_solve: the Jacobi-PCG workspace of a solve (residual,
// search direction, product, Jacobi inverse, their FP32 twins, partial sums, solver
// states) lives in one file-scope device array instead of a mesh handle's allocations,
// so the call allocates no device memory and needs no handle.
//
// Each GPU holds its own copy of the array (at its own address, taken once per device
// with hipGetSymbolAddress); every solve on a device works in that device's copy, which
// keeps the last call's contents.  Calls on one device are serialised by a lock (a call
// returns only when its solve has finished), so two of them never work in the array at
// the same time.
#include <cstring>
#include <mutex>

#include "solver.hpp"

namespace rafem {
namespace {

constexpr int64_t kMaxRows = RAFEM_NOALLOC_MAX_ROWS;
constexpr size_t kPartSlots = (size_t)kMaxRows / 64 + 64;  // as a mesh handle sizes them
constexpr size_t kMaxDevices = 64;

constexpr size_t up256(size_t x) { return (x + 255) & ~size_t(255); }
// byte offsets of the workspace vectors inside the array
constexpr size_t kVec64 = up256(8 * (size_t)kMaxRows), kVec32 = up256(4 * (size_t)kMaxRows);
constexpr size_t kOffR = 0, kOffP = kOffR + kVec64, kOffQ = kOffP + kVec64,
                 kOffDinv = kOffQ + kVec64, kOffR64 = kOffDinv + kVec64,
                 kOffR32 = kOffR64 + kVec64, kOffP32 = kOffR32 + kVec32,
                 kOffQ32 = kOffP32 + kVec32, kOffD32 = kOffQ32 + kVec32,
                 kOffDinv32 = kOffD32 + kVec32, kOffPartials = kOffDinv32 + kVec32,
                 kOffPartPq = kOffPartials + up256(3 * 8 * kPartSlots),
                 kOffPartRz = kOffPartPq + up256(8 * kPartSlots),
                 kOffStates = kOffPartRz + up256(2 * 8 * kPartSlots),
                 kOffItb = kOffStates + up256(3 * sizeof(PcgState)),
                 kOffRowOff = kOffItb + 256, kScratchBytes = kOffRowOff + 256;
static_assert(kScratchBytes == RAFEM_NOALLOC_SCRATCH_BYTES, "scratch size in rafem.h");

// The workspace of every allocation-free solve on a device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Row range {0, n} of the single system (the solver kernels locate a system's partial slots
// from it).
__global__ void k_noalloc_rows(int32_t* row_off, int32_t n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        row_off[0] = 0;
        row_off[1] = n;
    }
}

struct DeviceSlot {
    bool ready = false;
    unsigned char* base = nullptr;  // the device's copy of `scratch`
    rafem_mesh_s ws;                // the solver's view of the workspace
    PcgState host_states[3];        // host copies of the states (polls)
    std::mutex mu;
};
DeviceSlot g_slots[kMaxDevices];
std::mutex g_init_mu;

// Once per device, with that device current: the address of its copy of the array, and
// the workspace pointers into it.
DeviceSlot& slot_for_current_device() {
    int dev = 0;
    RAFEM_HIP(hipGetDevice(&dev));
    if (dev < 0 || (size_t)dev >= kMaxDevices)
        throw Error{RAFEM_E_ARG, "device ordinal beyond the allocation-free entry point's table"};
    DeviceSlot& d = g_slots[dev];
    std::lock_guard<std::mutex> lock(g_init_mu);
    if (d.ready) return d;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        throw Error{RAFEM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e)};
    unsigned char* b = static_cast<unsigned char*>(ptr);
    rafem_mesh_s& w = d.ws;
    w.device = dev;
    w.S = 1;
    w.r = reinterpret_cast<double*>(b + kOffR);
    w.p = reinterpret_cast<double*>(b + kOffP);
    w.q = reinterpret_cast<double*>(b + kOffQ);
    w.dinv = reinterpret_cast<double*>(b + kOffDinv);
    w.r64 = reinterpret_cast<double*>(b + kOffR64);
    w.r32 = reinterpret_cast<float*>(b + kOffR32);
    w.p32 = reinterpret_cast<float*>(b + kOffP32);
    w.q32 = reinterpret_cast<float*>(b + kOffQ32);
    w.d32 = reinterpret_cast<float*>(b + kOffD32);
    w.dinv32 = reinterpret_cast<float*>(b + kOffDinv32);
    w.partials = reinterpret_cast<double*>(b + kOffPartials);
    w.part_pq = reinterpret_cast<double*>(b + kOffPartPq);
    w.part_rz = reinterpret_cast<double*>(b + kOffPartRz);
    w.st = reinterpret_cast<PcgState*>(b + kOffStates);
    w.itb = reinterpret_cast<int32_t*>(b + kOffItb);
    w.row_off_one = reinterpret_cast<int32_t*>(b + kOffRowOff);
    w.row_off = w.row_off_one;
    w.st_host = d.host_states;
    w.use_graphs = false;
    w.prof_on = false;
    d.base = b;
    d.ready = true;
    return d;
}

}  // namespace
}  // namespace rafem

extern "C" rafem_status rafem_solve_noalloc(int64_t n_rows, int64_t nnz, const int32_t* row_ptr_d,
                                            const int32_t* col_idx_d, const double* vals_d,
                                            const float* vals32_d, const double* b_d,
                                            double* x_d, const rafem_solve_opts* opts,
                                            rafem_solve_info* info, void* stream) {
    using namespace rafem;
    try {
        clear_error();
        if (n_rows < 1 || n_rows > kMaxRows)
            throw Error{RAFEM_E_ARG, "n_rows must be in [1, RAFEM_NOALLOC_MAX_ROWS = " +
                                         std::to_string(kMaxRows) + "], got " +
                                         std::to_string(n_rows)};
        if (nnz < n_rows || nnz > INT32_MAX)
            throw Error{RAFEM_E_ARG, "nnz must be in [n_rows, INT32_MAX]"};
        if (!row_ptr_d || !col_idx_d || !vals_d || !b_d || !x_d)
            throw Error{RAFEM_E_ARG, "NULL matrix or vector argument"};
        SolveOpts o = resolve_opts(opts, 1e-10);
        if (o.precision == RAFEM_MIXED && !vals32_d)
            throw Error{RAFEM_E_ARG, "MIXED precision needs vals32"};
        DeviceSlot& d = slot_for_current_device();
        std::lock_guard<std::mutex> lock(d.mu);
        rafem_mesh_s& w = d.ws;
        w.n = n_rows;
        w.nnz = nnz;
        w.spmv = choose_spmv_config(n_rows, nnz);
        w.spmv32 = w.spmv;
        hipStream_t s = (hipStream_t)stream;
        hipLaunchKernelGGL(k_noalloc_rows, dim3(1), dim3(64), 0, s, w.row_off_one, (int32_t)n_rows);
        RAFEM_HIP(hipGetLastError());
        Mat A;
        A.n = (int32_t)n_rows;
        A.sell = 0;
        A.rp = row_ptr_d;
        A.ci = col_idx_d;
        A.v = vals_d;
        A.v32 = vals32_d;
        const Samples one{1, w.row_off_one};
        const rafem_status st =
            o.precision == RAFEM_MIXED
                ? pcg_mixed(&w, A, one, nullptr, nullptr, b_d, x_d, o, info, s, nullptr)
                : pcg64(&w, A, one, nullptr, b_d, x_d, o, info, s, nullptr);
        if (st != RAFEM_OK)
            set_error(st == RAFEM_E_NOCONV ? "iteration limit reached"
                                           : "PCG breakdown (p.Ap <= 0 or non-finite)");
        return st;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return RAFEM_E_HIP;
    } catch (...) {
        set_error("unknown error");
        return RAFEM_E_HIP;
    }
}
