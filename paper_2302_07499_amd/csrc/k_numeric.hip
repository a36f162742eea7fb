// Numeric phase: per-pair inner integrals (fullcaps), reduction of each outer
// tet's contributions in LDS, the inner-element terms, the sorted-key
// segmented sums into the CSR values and the right-hand side.
//
// Decomposition of the pair contribution (main assembly algorithm, Sec. 4.3):
// with a_u(y) = phi_(m,u)(y) - phi_(n,u)(p) and the moments S0, S1, S2 of the
// inner tet's barycentric coordinates over E_m n B_{delta,h}(p),
//   K_uv = f_m psi w [S2_uv - c_u S1_v - c_v S1_u + c_u c_v S0]
// (c = the outer rule row of p, f_m = 1 on T_Omega, 2 on T_OmegaI).  Summed
// over the pairs, the c c^T S0 terms only need T0_k = sum_m f_m S0 per outer
// point, the cross terms only R_k(v) = sum_{m containing v} f_m S1_v per
// (outer point, vertex), and the S2 terms only the per-inner-tet sum
// G_m = sum_q psi f_m w_q S2.  The first two are reduced inside the outer
// tet's workgroup, G_m through a buffer ordered by inner tet.
#include "device_geom.hpp"

#ifndef NLFEM_INTEGRATE_WAVES
#define NLFEM_INTEGRATE_WAVES 3  // minimum waves per SIMD requested for k_integrate (register cap)
#endif

namespace nlfem {

namespace {

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int32_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Non-negative x is added to a two-word fixed-point sum: the coarse word
// counts units of 2^-s, the fine word the remainder in units of 2^-(s+48).
// Integer sums are order-independent, so the result is deterministic, and the
// fine word keeps small contributions (thin cut slivers) relatively exact.
constexpr int FX_LO_BITS = 48;

__device__ __forceinline__ void fx_add(unsigned long long* hi, unsigned long long* lo, double x, double fx) {
    const double xs = x * fx;  // exact: fx is a power of two
    const double h = floor(xs);
    const double r = xs - h;   // exact, in [0, 1)
    atomicAdd(hi, (unsigned long long)h);
    atomicAdd(lo, (unsigned long long)__double2ull_rn(r * 281474976710656.0));  // r * 2^48
}

__device__ __forceinline__ double fx_value(unsigned long long hi, unsigned long long lo, int shift) {
    return (double)hi * ldexp(1.0, -shift) + (double)lo * ldexp(1.0, -(shift + FX_LO_BITS));
}

// One workgroup of BLOCK threads integrates one outer tet.  LDS: R [4][umax]
// and T0 [4] as two-word fixed-point sums (coarse words, then fine words),
// Ve [umax], and the 4 outer points.
template <typename T, int BLOCK>
__device__ __forceinline__ void integrate_outer(const IntegrateArgs& a, int64_t oi, unsigned long long* smem64,
                                                double (*P)[3]) {
    const int umax = a.umax;
    unsigned long long* R = smem64;             // coarse [4][umax]
    unsigned long long* Rl = R + 4 * umax;      // fine   [4][umax]
    unsigned long long* T0 = Rl + 4 * umax;     // coarse [4]
    unsigned long long* T0l = T0 + 4;           // fine   [4]
    int32_t* ve = (int32_t*)(T0l + 4);
    const int n = a.outer_ids[oi];
    const int64_t vb = a.ve_off[oi];
    const int U = (int)(a.ve_off[oi + 1] - vb);
    const int t = threadIdx.x;
    for (int i = t; i < U; i += BLOCK) ve[i] = a.ve_ids[vb + i];
    for (int i = t; i < 8 * umax; i += BLOCK) R[i] = 0ull;
    if (t < 4) {
        T0[t] = 0ull;
        T0l[t] = 0ull;
        double Xn[12];
        for (int i = 0; i < 12; ++i) Xn[i] = a.tetX[12 * (int64_t)n + i];
        outer_point(Xn, t, P[t]);
    }
    const double w = a.vol[n] * 0.25;
    __syncthreads();
    const double d2 = a.delta * a.delta;
    const double fx = ldexp(1.0, a.fx_shift);
    const int64_t p0 = a.pair_off[oi], p1 = a.pair_off[oi + 1];
    for (int64_t p = p0 + t; p < p1; p += BLOCK) {
        const int m = a.pair_m[p];
        const uint32_t code = a.pair_cls[p];
        double X[12];
        for (int i = 0; i < 12; ++i) X[i] = a.tetX[12 * (int64_t)m + i];
        const double volm = a.vol[m];
        const bool omega = a.region[m] != 0;
        const double fm = omega ? 1.0 : 2.0;
        int lv[4];
        for (int j = 0; j < 4; ++j) lv[j] = lower_bound_i32(ve, U, a.tets[4 * (int64_t)m + j]);
        double g[10];
        for (int i = 0; i < 10; ++i) g[i] = 0.0;
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int c = (int)((code >> (3 * k)) & 7u);
            if (c == C_OUT) continue;
            double S[15];
            pair_moments<T>(X, volm, P[k], d2, c, a.mc_samples, a.key0, a.key1, (uint32_t)(4 * n + k), (uint32_t)m,
                            S);
            fx_add(&T0[k], &T0l[k], fm * S[0], fx);
            for (int j = 0; j < 4; ++j)
                if (lv[j] < U)  // always true: Ve holds every vertex of the pair list's tets
                    fx_add(&R[k * umax + lv[j]], &Rl[k * umax + lv[j]], fm * S[1 + j], fx);
            for (int i = 0; i < 10; ++i) g[i] += S[5 + i];
        }
        if (omega) {
            double* gb = a.g_buf + 10 * (size_t)a.tpos[p];
            const double sc = a.psi * w;
            for (int i = 0; i < 10; ++i) gb[i] = g[i] * sc;
        }
    }
    __syncthreads();
    const double pw = a.psi * w;
    const int sh = a.fx_shift;
    int32_t vn[4];
    for (int j = 0; j < 4; ++j) vn[j] = a.tets[4 * (int64_t)n + j];
    double t0[4];
    for (int k = 0; k < 4; ++k) t0[k] = fx_value(T0[k], T0l[k], sh);
    const int64_t rb = a.rec_off[oi];
    // direct rows u = V_n[j], columns Ve[i]: psi w (sum_k c_u c_v T0_k [v in V_n] - sum_k c_u R_k(v))
    for (int r = t; r < 4 * U; r += BLOCK) {
        const int j = r / U, i = r - j * U;
        double cR = 0.0;
        for (int k = 0; k < 4; ++k) cR += rule_w(k, j) * fx_value(R[k * umax + i], Rl[k * umax + i], sh);
        const int32_t v = ve[i];
        double O = 0.0;
        for (int jj = 0; jj < 4; ++jj)
            if (vn[jj] == v)
                for (int k = 0; k < 4; ++k) O += (rule_w(k, j) * rule_w(k, jj)) * t0[k];
        a.rec_val[rb + r] = pw * (O - cR);
    }
    // transposed rows Ve[i], columns u = V_n[j]: the cross term again
    for (int r = t; r < 4 * U; r += BLOCK) {
        const int i = r >> 2, j = r & 3;
        double cR = 0.0;
        for (int k = 0; k < 4; ++k) cR += rule_w(k, j) * fx_value(R[k * umax + i], Rl[k * umax + i], sh);
        a.rec_val[rb + 4 * (int64_t)U + r] = -(pw * cR);
    }
    // load vector: sum_k w c_u f(p_k)
    if (t < 4) {
        double f = 0.0;
        if (a.f_qp)
            for (int k = 0; k < 4; ++k) f += (w * rule_w(k, t)) * a.f_qp[4 * (int64_t)n + k];
        a.rec_val[rb + 8 * (int64_t)U + t] = f;
    }
}

template <typename T>
__global__ __launch_bounds__(256, NLFEM_INTEGRATE_WAVES) void k_integrate(IntegrateArgs a) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    integrate_outer<T, 256>(a, (int64_t)blockIdx.x, smem64, P);
}

// Persistent batched integration: every workgroup takes work items (mesh,
// outer tet) from a device queue until it is empty.  Items are ordered by
// decreasing estimated cost; each item's results depend on the item only.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK, NLFEM_INTEGRATE_WAVES) void k_integrate_batch(const IntegrateArgs* descs, const int2* items,
                                                           int64_t n_items, unsigned long long* head) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    __shared__ long long cur;
    while (true) {
        if (threadIdx.x == 0) cur = (long long)atomicAdd(head, 1ull);
        __syncthreads();
        const long long it = cur;
        __syncthreads();
        if (it >= n_items) break;
        const int2 item = items[it];
        integrate_outer<T, BLOCK>(descs[item.x], (int64_t)item.y, smem64, P);
        __syncthreads();
    }
}

__global__ void k_reset_u64(unsigned long long* p) { *p = 0ull; }

// per-pair moments for outer positions [o_lo, o_hi): slot (p - pair_off[o_lo])*4 + k
template <typename T>
__global__ __launch_bounds__(256) void k_debug_pairs(IntegrateArgs a, int64_t o_lo, double* out_S, int32_t* out_qm) {
    const int64_t oi = o_lo + blockIdx.x;
    const int n = a.outer_ids[oi];
    double Xn[12];
    for (int i = 0; i < 12; ++i) Xn[i] = a.tetX[12 * (int64_t)n + i];
    double P[4][3];
    for (int k = 0; k < 4; ++k) outer_point(Xn, k, P[k]);
    const double d2 = a.delta * a.delta;
    const int64_t base = a.pair_off[o_lo];
    for (int64_t p = a.pair_off[oi] + threadIdx.x; p < a.pair_off[oi + 1]; p += 256) {
        const int m = a.pair_m[p];
        const uint32_t code = a.pair_cls[p];
        double X[12];
        for (int i = 0; i < 12; ++i) X[i] = a.tetX[12 * (int64_t)m + i];
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int c = (int)((code >> (3 * k)) & 7u);
            const int64_t idx = (p - base) * 4 + k;
            out_qm[3 * idx] = 4 * n + k;
            out_qm[3 * idx + 1] = m;
            out_qm[3 * idx + 2] = c;
            if (c == C_OUT) continue;
            double S[15];
            pair_moments<T>(X, a.vol[m], P[k], d2, c, a.mc_samples, a.key0, a.key1, (uint32_t)(4 * n + k),
                            (uint32_t)m, S);
            for (int i = 0; i < 15; ++i) out_S[15 * idx + i] = S[i];
        }
    }
}

__device__ __forceinline__ int tri4(int a, int b) {
    // upper-triangle index of (a,b), a <= b: 00 01 02 03 11 12 13 22 23 33
    const int rowstart[4] = {0, 4, 7, 9};
    return rowstart[a] + (b - a);
}

// G_m = sum over the pairs (n, m) in transposed order; records [16] per tet
__global__ void k_g_reduce(const uint8_t* region, int64_t K, const int64_t* trans_off, const double* g_buf,
                           int64_t rec_base, double* rec_val) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const int64_t b = trans_off[e], c = trans_off[e + 1];
    if (!region[e] || c <= b) return;
    double G[10];
    for (int j = 0; j < 10; ++j) G[j] = 0.0;
    for (int64_t i = b; i < c; ++i)
        for (int j = 0; j < 10; ++j) G[j] += g_buf[10 * i + j];
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) rec_val[rec_base + 16 * e + 4 * x + y] = G[x <= y ? tri4(x, y) : tri4(y, x)];
}

__global__ void k_segsum(const int64_t* seg_off, const uint32_t* perm, const double* rec_val, int64_t n_slots,
                         const int64_t* dest, int64_t nnz_ff, int64_t nnz_fc, double* ff_val, double* fc_val,
                         double* rhs_f) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    double acc = 0.0;
    for (int64_t i = seg_off[s]; i < seg_off[s + 1]; ++i) acc += rec_val[perm[i]];
    const int64_t d = dest[s];
    if (d < nnz_ff) ff_val[d] = acc;
    else if (d < nnz_ff + nnz_fc) fc_val[d - nnz_ff] = acc;
    else rhs_f[d - nnz_ff - nnz_fc] = acc;
}

__global__ void k_rhs_final(int64_t n_free, const double* rhs_f, const int64_t* fc_row_ptr, const int32_t* fc_col,
                            const double* fc_val, const double* g, double* rhs) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_free) return;
    double acc = 0.0;
    if (g)
        for (int64_t e = fc_row_ptr[r]; e < fc_row_ptr[r + 1]; ++e) acc = acc + fc_val[e] * g[fc_col[e]];
    rhs[r] = rhs_f[r] - acc;
}

__global__ void k_fill_zero(double* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
__global__ void k_copy_i64(const int64_t* a, int64_t* b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
__global__ void k_copy_i32(const int32_t* a, int32_t* b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_class_counts(const uint16_t* pair_cls, int64_t P, unsigned long long* counts) {
    __shared__ unsigned long long c[6];
    if (threadIdx.x < 6) c[threadIdx.x] = 0ull;
    __syncthreads();
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        uint32_t code = pair_cls[p];
        for (int k = 0; k < 4; ++k) {
            unsigned cl = (code >> (3 * k)) & 7u;
            if (cl != 0u) atomicAdd(&c[cl], 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) atomicAdd(&counts[threadIdx.x], c[threadIdx.x]);
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t integrate_lds_bytes(int umax) { return (size_t)umax * 68 + 64; }

hipError_t launch_integrate(const IntegrateArgs& a, bool fp32, hipStream_t s) {
    if (a.n_outer <= 0) return hipSuccess;
    size_t sh = integrate_lds_bytes(a.umax);
    if (fp32) k_integrate<float><<<(unsigned)a.n_outer, 256, sh, s>>>(a);
    else k_integrate<double><<<(unsigned)a.n_outer, 256, sh, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_integrate_batch(const IntegrateArgs* descs, const int2* items, int64_t n_items,
                                  unsigned long long* head, int umax, bool fp32, int block, int grid, hipStream_t s) {
    size_t sh = integrate_lds_bytes(umax);
    k_reset_u64<<<1, 1, 0, s>>>(head);
    if (n_items <= 0) return hipGetLastError();
    if (block == 128) {
        if (fp32) k_integrate_batch<float, 128><<<grid, 128, sh, s>>>(descs, items, n_items, head);
        else k_integrate_batch<double, 128><<<grid, 128, sh, s>>>(descs, items, n_items, head);
    } else {
        if (fp32) k_integrate_batch<float, 256><<<grid, 256, sh, s>>>(descs, items, n_items, head);
        else k_integrate_batch<double, 256><<<grid, 256, sh, s>>>(descs, items, n_items, head);
    }
    return hipGetLastError();
}

hipError_t launch_debug_pairs(const IntegrateArgs& a, bool fp32, int64_t o_lo, int64_t o_hi, double* out_S,
                              int32_t* out_qm, hipStream_t s) {
    if (o_hi <= o_lo) return hipSuccess;
    if (fp32) k_debug_pairs<float><<<(unsigned)(o_hi - o_lo), 256, 0, s>>>(a, o_lo, out_S, out_qm);
    else k_debug_pairs<double><<<(unsigned)(o_hi - o_lo), 256, 0, s>>>(a, o_lo, out_S, out_qm);
    return hipGetLastError();
}

hipError_t launch_g_reduce(const uint8_t* region, int64_t K, const int64_t* trans_off, const double* g_buf,
                           int64_t rec_base, double* rec_val, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_g_reduce<<<blocks_for(K), 256, 0, s>>>(region, K, trans_off, g_buf, rec_base, rec_val);
    return hipGetLastError();
}

hipError_t launch_segsum(const int64_t* seg_off, const uint32_t* perm, const double* rec_val, int64_t n_slots,
                         const int64_t* dest, int64_t nnz_ff, int64_t nnz_fc, double* ff_val, double* fc_val,
                         double* rhs_f, hipStream_t s) {
    if (n_slots <= 0) return hipSuccess;
    k_segsum<<<blocks_for(n_slots), 256, 0, s>>>(seg_off, perm, rec_val, n_slots, dest, nnz_ff, nnz_fc, ff_val,
                                                 fc_val, rhs_f);
    return hipGetLastError();
}

hipError_t launch_rhs_final(int64_t n_free, const double* rhs_f, const int64_t* fc_row_ptr, const int32_t* fc_col,
                            const double* fc_val, const double* g, double* rhs, hipStream_t s) {
    if (n_free <= 0) return hipSuccess;
    k_rhs_final<<<blocks_for(n_free), 256, 0, s>>>(n_free, rhs_f, fc_row_ptr, fc_col, fc_val, g, rhs);
    return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_zero<<<blocks_for(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_copy_i64<<<blocks_for(n), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_copy_i32<<<blocks_for(n), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_class_counts(const uint16_t* pair_cls, int64_t P, unsigned long long* counts, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    int64_t b = (P + 255) / 256;
    if (b > 2048) b = 2048;
    k_class_counts<<<(unsigned)b, 256, 0, s>>>(pair_cls, P, counts);
    return hipGetLastError();
}

}  // namespace nlfem
