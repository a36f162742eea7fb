// Device-wide exclusive scan (int64) and stable LSD radix sort of
// (uint64 key, uint32 value) pairs, 8-bit digits, wave64 ballot ranking.
#include "common.hpp"

namespace nlfem {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int64_t block_scan_excl(int64_t v, int64_t* sh, int64_t* total) {
    // Hillis-Steele over 256 values in shared memory (deterministic order)
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int64_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_block_sums(const int64_t* in, int64_t n, int64_t* sums) {
    __shared__ int64_t sh[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) acc += in[idx];
    }
    int64_t tot;
    block_scan_excl(acc, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_block_scan(const int64_t* in, int64_t n, const int64_t* offs,
                                                            int64_t* out, int write_total) {
    __shared__ int64_t sh[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t v[SCAN_ITEMS];
    int64_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        v[i] = (idx < n) ? in[idx] : 0;
        acc += v[i];
    }
    int64_t tot;
    int64_t pre = block_scan_excl(acc, sh, &tot);
    int64_t o = offs ? offs[blockIdx.x] : 0;
    int64_t run = o + pre;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_ITEMS + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) out[n] = o + tot;
}

int64_t nblocks(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    size_t b = 0;
    int64_t m = n;
    while (true) {
        int64_t nb = nblocks(m);
        b += (size_t)(nb + 1) * 2 * sizeof(int64_t);
        if (nb <= 1) break;
        m = nb;
    }
    return b + 256;
}

// out has n+1 entries; out[n] = total.  temp: scan_temp_bytes(n)
namespace {
__global__ void k_zero1(int64_t* p) { *p = 0; }
}  // namespace

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp, hipStream_t s) {
    if (n <= 0) {
        k_zero1<<<1, 1, 0, s>>>(out);
        return hipGetLastError();
    }
    int64_t nb = nblocks(n);
    if (nb == 1) {
        k_block_scan<<<1, SCAN_BLOCK, 0, s>>>(in, n, nullptr, out, 1);
        return hipGetLastError();
    }
    int64_t* sums = (int64_t*)temp;
    int64_t* sums_scan = sums + (nb + 1);
    void* rest = (void*)(sums_scan + (nb + 1));
    k_block_sums<<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_i64(sums, sums_scan, nb, rest, s);
    if (e != hipSuccess) return e;
    k_block_scan<<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, sums_scan, out, 1);
    return hipGetLastError();
}

namespace {
__global__ void k_u8_to_i64(const uint8_t* in, int64_t n, int64_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] ? 1 : 0;
}
__global__ void k_i64_to_i32(const int64_t* in, int64_t n, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) out[i] = (int32_t)in[i];
}
}  // namespace

hipError_t exclusive_scan_u8_to_i32(const uint8_t* in, int32_t* out, int64_t n, void* temp, hipStream_t s) {
    int64_t* a = (int64_t*)temp;
    int64_t* b = a + (n + 1);
    void* rest = (void*)(b + (n + 2));
    if (n > 0) {
        k_u8_to_i64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, n, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e = exclusive_scan_i64(a, b, n, rest, s);
    if (e != hipSuccess) return e;
    k_i64_to_i32<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(b, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
namespace {
constexpr int RS_BLOCK = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ROUNDS;

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t* keys, int64_t n, int shift, int64_t n_tiles,
                                                      int64_t* hist) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + (int64_t)r * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t* keys, const uint32_t* vals, int64_t n,
                                                         int shift, int64_t n_tiles, const int64_t* offs,
                                                         uint64_t* okeys, uint32_t* ovals) {
    __shared__ int64_t running[256];
    __shared__ int wcount[4][256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    running[t] = offs[(int64_t)t * n_tiles + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        for (int w = 0; w < 4; ++w) wcount[w][t] = 0;
        __syncthreads();
        int64_t i = base + (int64_t)r * RS_BLOCK + t;
        bool valid = i < n;
        uint64_t k = valid ? keys[i] : 0;
        uint32_t v = valid ? vals[i] : 0;
        unsigned d = (unsigned)((k >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcount[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t pos = running[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][d];
            okeys[pos] = k;
            ovals[pos] = v;
        }
        __syncthreads();
        running[t] += (int64_t)wcount[0][t] + wcount[1][t] + wcount[2][t] + wcount[3][t];
        __syncthreads();
    }
}
}  // namespace

size_t radix_sort_temp_bytes(int64_t n) {
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    int64_t h = tiles * 256;
    return (size_t)(2 * (h + 1)) * sizeof(int64_t) + scan_temp_bytes(h) + 256;
}

hipError_t radix_sort_u64_u32(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals, int64_t n,
                              int nbits, void* temp, hipStream_t s) {
    if (n <= 1 || nbits <= 0) return hipSuccess;
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    int64_t h = tiles * 256;
    int64_t* hist = (int64_t*)temp;
    int64_t* offs = hist + (h + 1);
    void* stemp = (void*)(offs + (h + 1));
    int passes = (nbits + 7) / 8;
    uint64_t *ki = keys, *ko = alt_keys;
    uint32_t *vi = vals, *vo = alt_vals;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_rs_hist<<<(unsigned)tiles, RS_BLOCK, 0, s>>>(ki, n, shift, tiles, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan_i64(hist, offs, h, stemp, s);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<(unsigned)tiles, RS_BLOCK, 0, s>>>(ki, vi, n, shift, tiles, offs, ko, vo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    if (ki != keys) {
        hipError_t e = hipMemcpyAsync(keys, ki, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, vi, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
__global__ void k_reduce_max(const int64_t* in, int64_t n, long long* out) {
    __shared__ long long sh[256];
    long long m = LLONG_MIN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (long long)in[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sh[0]);
}
__global__ void k_set_i64(long long* p, long long v) { *p = v; }
}  // namespace

hipError_t reduce_max_i64(const int64_t* in, int64_t n, int64_t* out_dev, hipStream_t s) {
    k_set_i64<<<1, 1, 0, s>>>((long long*)out_dev, 0);
    if (n <= 0) return hipGetLastError();
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    k_reduce_max<<<(unsigned)blocks, 256, 0, s>>>(in, n, (long long*)out_dev);
    return hipGetLastError();
}

}  // namespace nlfem
