// FP64 conjugate-gradient building blocks: CSR SpMV (one wave per row),
// deterministic two-level dot products, and the vector updates with the
// step lengths kept on the device.
#include "common.hpp"

namespace nlfem {

namespace {

constexpr int DOT_BLOCKS = 512;

__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* va,
                                              const double* x, double* y) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += 64) acc += va[e] * x[ci[e]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = acc;
}

__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* a, const double* b, double* partial) {
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

__global__ __launch_bounds__(256) void k_dot_final(const double* partial, double* out) {
    __shared__ double sh[256];
    sh[threadIdx.x] = partial[threadIdx.x] + partial[threadIdx.x + 256];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_cg_init(int64_t n, const double* b, const double* Ax, double* r, double* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = b[i] - Ax[i];
    r[i] = v;
    p[i] = v;
}

__global__ void k_cg_xr(int64_t n, const double* sc, double* x, double* r, const double* p, const double* Ap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = sc[0] / sc[1];
    x[i] = x[i] + alpha * p[i];
    r[i] = r[i] - alpha * Ap[i];
}

__global__ void k_cg_p(int64_t n, const double* sc, const double* r, double* p) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = sc[2] / sc[0];
    p[i] = r[i] + beta * p[i];
}

__global__ void k_copy1(const double* a, double* b) { *b = *a; }

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* x, double* y,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_spmv<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(n, rp, ci, va, x, y);
    return hipGetLastError();
}

// partial must hold DOT_BLOCKS doubles
hipError_t launch_dot(int64_t n, const double* a, const double* b, double* partial, double* out, hipStream_t s) {
    k_dot_partial<<<DOT_BLOCKS, 256, 0, s>>>(n, a, b, partial);
    k_dot_final<<<1, 256, 0, s>>>(partial, out);
    return hipGetLastError();
}

hipError_t launch_cg_init(int64_t n, const double* b, const double* Ax, double* x, double* r, double* p,
                          hipStream_t s) {
    (void)x;
    if (n <= 0) return hipSuccess;
    k_cg_init<<<blocks_for(n), 256, 0, s>>>(n, b, Ax, r, p);
    return hipGetLastError();
}

hipError_t launch_cg_xr(int64_t n, const double* sc, double* x, double* r, const double* p, const double* Ap,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cg_xr<<<blocks_for(n), 256, 0, s>>>(n, sc, x, r, p, Ap);
    return hipGetLastError();
}

hipError_t launch_cg_p(int64_t n, double* sc, const double* r, double* p, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cg_p<<<blocks_for(n), 256, 0, s>>>(n, sc, r, p);
    k_copy1<<<1, 1, 0, s>>>(sc + 2, sc);
    return hipGetLastError();
}

hipError_t launch_copy_scalar(const double* src, double* dst, hipStream_t s) {
    k_copy1<<<1, 1, 0, s>>>(src, dst);
    return hipGetLastError();
}

}  // namespace nlfem
