// FP64 conjugate gradients for the free-node system (the CG solve that ends
// the main assembly algorithm, Sec. 4.3): CSR SpMV (one wave per row),
// deterministic two-level dot products, and the vector updates.  The scalars
// (step lengths, residual norms) and the stopping decision stay on the device
// in a CgState, so the host only polls it every few iterations: every kernel
// of an iteration returns at once when the state says the solve has stopped,
// which keeps the iteration count exact however many iterations are queued.
//
// The work vectors come from the caller: a scratch block of cg_work_doubles(n)
// doubles, either allocated by the library (nlfem_cg) or the file-scope
// device array below (nlfem_cg_noalloc, for callers that cannot allocate).
#include <mutex>

#include "common.hpp"

namespace nlfem {

namespace {

constexpr int DOT_BLOCKS = 512;

// Device scratch of the allocation-free CG: r, p, Ap for up to kCgNoAllocMaxN
// rows, the dot partials and the state.  One copy per GPU, held until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) static double scratch[3 * (size_t)kCgNoAllocMaxN + DOT_BLOCKS + 64];

// done: 0 running, 1 converged, 2 breakdown (p.Ap <= 0 or a non-finite
// value), 3 iteration cap reached, 4 zero right-hand side
__device__ __forceinline__ bool stopped(const CgState* st) { return *(volatile const int*)&st->done != 0; }

__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* va,
                                              const double* x, double* y, const CgState* st) {
    if (st && stopped(st)) return;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += 64) acc += va[e] * x[ci[e]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = acc;
}

__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* a, const double* b, double* partial,
                                                     const CgState* st) {
    if (st && stopped(st)) return;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)DOT_BLOCKS * 256)
        acc += a[i] * b[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// sum of the DOT_BLOCKS partials in a fixed order (the same value in every
// block that calls it); needs blockDim.x == 256
__device__ __forceinline__ double dot_total(const double* partial, double* sh) {
    sh[threadIdx.x] = partial[threadIdx.x] + partial[threadIdx.x + 256];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double v = sh[0];
    __syncthreads();
    return v;
}

__global__ __launch_bounds__(256) void k_dot_final(const double* partial, double* out) {
    __shared__ double sh[256];
    const double v = dot_total(partial, sh);
    if (threadIdx.x == 0) *out = v;
}

__global__ void k_cg_init(int64_t n, const double* b, const double* Ax, double* r, double* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = b[i] - Ax[i];
    r[i] = v;
    p[i] = v;
}

// after the initial residual: the threshold rtol ||b||, and whether the
// start vector already meets it (the same IEEE operations the loop uses)
__global__ void k_cg_begin(CgState* st, double rtol, int max_iter) {
    const double bn = sqrt(st->bb);
    st->bnorm = bn;
    st->thr = rtol * bn;
    st->res2 = st->rr[0];
    st->pAp = 0.0;
    st->iter = 0;
    st->max_iter = max_iter;
    if (bn == 0.0) st->done = 4;
    else if (sqrt(st->rr[0]) <= st->thr) st->done = 1;
    else if (max_iter <= 0) st->done = 3;
    else st->done = 0;
}

// iteration it: pAp from the partials, alpha = rr_it / pAp, x += alpha p,
// r -= alpha Ap.  Every block forms the same alpha.
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int it, CgState* st, const double* partial, double* x,
                                               double* r, const double* p, const double* Ap) {
    if (stopped(st)) return;
    __shared__ double sh[256];
    const double pAp = dot_total(partial, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->pAp = pAp;
    const double alpha = st->rr[it & 1] / pAp;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x[i] = x[i] + alpha * p[i];
        r[i] = r[i] - alpha * Ap[i];
    }
}

// end of iteration it: rr_{it+1} from the partials, the stopping decision
// (taken by every block alike, recorded by block 0), then p = r + beta p
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int it, CgState* st, const double* partial, const double* r,
                                              double* p) {
    if (stopped(st)) return;
    __shared__ double sh[256];
    const double rr1 = dot_total(partial, sh);
    const double rr0 = st->rr[it & 1];
    const double pAp = st->pAp;
    int done = 0;
    if (!(pAp > 0.0) || !isfinite(pAp) || !isfinite(rr1)) done = 2;
    else if (sqrt(rr1) <= st->thr) done = 1;
    else if (it + 1 >= st->max_iter) done = 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr[(it + 1) & 1] = rr1;
        st->res2 = rr1;
        st->iter = it + 1;
        st->done = done;
    }
    if (done) return;
    const double beta = rr1 / rr0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = r[i] + beta * p[i];
}

__global__ void k_zero(int64_t n, double* x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// grid of the vector updates: grid-stride, at most 1024 workgroups
inline unsigned update_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t cg_work_doubles(int64_t n) { return (size_t)3 * (size_t)n + DOT_BLOCKS + 64; }

hipError_t cg_noalloc_setup(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

void* cg_noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

hipError_t launch_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* x, double* y,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_spmv<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, rp, ci, va, x, y, nullptr);
    return hipGetLastError();
}

hipError_t cg_enqueue_start(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* b,
                            double* x, double rtol, int max_iter, double* work, hipStream_t s) {
    double* r = work;
    double* p = r + n;
    double* Ap = p + n;
    double* partial = Ap + n;
    CgState* st = (CgState*)(partial + DOT_BLOCKS);
    k_spmv<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, rp, ci, va, x, Ap, nullptr);
    k_cg_init<<<blocks_for(n), 256, 0, s>>>(n, b, Ap, r, p);
    k_dot_partial<<<DOT_BLOCKS, 256, 0, s>>>(n, r, r, partial, nullptr);
    k_dot_final<<<1, 256, 0, s>>>(partial, &st->rr[0]);
    k_dot_partial<<<DOT_BLOCKS, 256, 0, s>>>(n, b, b, partial, nullptr);
    k_dot_final<<<1, 256, 0, s>>>(partial, &st->bb);
    k_cg_begin<<<1, 1, 0, s>>>(st, rtol, max_iter);
    return hipGetLastError();
}

hipError_t cg_enqueue_iterations(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, double* x,
                                 int it0, int count, double* work, hipStream_t s) {
    double* r = work;
    double* p = r + n;
    double* Ap = p + n;
    double* partial = Ap + n;
    CgState* st = (CgState*)(partial + DOT_BLOCKS);
    const unsigned ub = update_blocks(n);
    for (int it = it0; it < it0 + count; ++it) {
        k_spmv<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, rp, ci, va, p, Ap, st);
        k_dot_partial<<<DOT_BLOCKS, 256, 0, s>>>(n, p, Ap, partial, st);
        k_cg_xr<<<ub, 256, 0, s>>>(n, it, st, partial, x, r, p, Ap);
        k_dot_partial<<<DOT_BLOCKS, 256, 0, s>>>(n, r, r, partial, st);
        k_cg_p<<<ub, 256, 0, s>>>(n, it, st, partial, r, p);
    }
    return hipGetLastError();
}

hipError_t cg_enqueue_zero(int64_t n, double* x, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zero<<<blocks_for(n), 256, 0, s>>>(n, x);
    return hipGetLastError();
}

const CgState* cg_state(const double* work, int64_t n) { return (const CgState*)(work + 3 * n + DOT_BLOCKS); }

}  // namespace nlfem
