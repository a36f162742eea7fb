// Row-wise assembly of the CSR system from the per-outer-tet results.
//
// For a free vertex u, the row A_u. collects (main assembly algorithm,
// Sec. 4.3, with the pair contribution split as in k_numeric.hip):
//  * direct terms of every outer tet n containing u: its cross block
//    C^n[j(u)][.] over the ball vertex set Ve_n, plus the outer-outer block
//    O^n[j(u)][.] on V_n;
//  * transposed terms of every outer tet n whose ball vertex set contains u:
//    C^n[j][i(u)] for the 4 columns V_n[j] (A is symmetric);
//  * inner-element terms G_m[a(u)][.] of every T_Omega tet m containing u;
//  * the load vector sum over outer tets n containing u of w c_u f.
// The sources of a row are found through two key-sorted lists built in the
// plan: vertex -> tets (all tets, stable by tet id) and vertex -> positions in
// the ball vertex sets.  The row's values are summed in LDS as two-word
// fixed point (order-independent, hence deterministic).
#include "common.hpp"

namespace nlfem {

namespace {

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__global__ void k_vt_keys(const int32_t* tets, int64_t K, uint64_t* keys, uint32_t* vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * K) return;
    keys[i] = (uint64_t)tets[i];
    vals[i] = (uint32_t)i;  // 4 * tet + local index
}

// off[k] = first sorted position with key >= k, off[n_keys] = n
__global__ void k_offsets(const uint64_t* skeys, int64_t n, int64_t n_keys, int64_t* off) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t prev = (i == 0) ? -1 : (int64_t)skeys[i - 1];
    int64_t cur = (i == n) ? n_keys : (int64_t)skeys[i];
    for (int64_t c = prev + 1; c <= cur; ++c) off[c] = i;
}

// incidence keys: ball vertex set entry g -> (vertex, g); owner[g] = outer position
__global__ void k_inc_keys(const int64_t* ve_off, int64_t n_outer, const int32_t* ve_ids, uint64_t* keys,
                           uint32_t* vals, int32_t* owner) {
    const int64_t oi = blockIdx.x;
    if (oi >= n_outer) return;
    for (int64_t g = ve_off[oi] + threadIdx.x; g < ve_off[oi + 1]; g += blockDim.x) {
        keys[g] = (uint64_t)ve_ids[g];
        vals[g] = (uint32_t)g;
        owner[g] = (int32_t)oi;
    }
}

// Pairs per inner tet.  A block takes kInnerGroup consecutive outer tets (mesh
// order: neighbours, whose balls share most of their inner tets), counts their
// inner tets in an LDS hash and adds each distinct count to inner_cnt once,
// instead of one global atomic per pair from blocks that all hit the same
// inner tets at the same time (the device-wide atomics are what this kernel
// waits on: 16 outer tets per block measured faster than 8 or 32); an inner
// tet that finds no slot within kInnerProbe probes is added directly.  The
// counts are exact either way.
constexpr int kInnerGroup = 16, kInnerHash = 4096, kInnerProbe = 32;
__global__ __launch_bounds__(256) void k_inner_count(const int64_t* pair_off, int64_t n_outer, const int32_t* pair_m,
                                                     int32_t* inner_cnt) {
    __shared__ int32_t key[kInnerHash];
    __shared__ int32_t cnt[kInnerHash];
    for (int i = threadIdx.x; i < kInnerHash; i += blockDim.x) {
        key[i] = -1;
        cnt[i] = 0;
    }
    __syncthreads();
    const int64_t o0 = (int64_t)blockIdx.x * kInnerGroup;
    const int64_t o1 = o0 + kInnerGroup < n_outer ? o0 + kInnerGroup : n_outer;
    const int64_t p1 = pair_off[o1];
    for (int64_t p = pair_off[o0] + threadIdx.x; p < p1; p += blockDim.x) {
        const int32_t m = pair_m[p];
        uint32_t h = ((uint32_t)m * 2654435761u) & (kInnerHash - 1);
        bool done = false;
        for (int k = 0; k < kInnerProbe && !done; ++k) {
            const int32_t prev = atomicCAS(&key[h], -1, m);
            if (prev == -1 || prev == m) {
                atomicAdd(&cnt[h], 1);
                done = true;
            }
            h = (h + 1) & (kInnerHash - 1);
        }
        if (!done) atomicAdd(&inner_cnt[m], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kInnerHash; i += blockDim.x)
        if (key[i] >= 0) atomicAdd(&inner_cnt[key[i]], cnt[i]);
}

__global__ void k_outer_pos(const int32_t* outer_ids, int64_t n_outer, int32_t* outer_pos) {
    int64_t oi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (oi < n_outer) outer_pos[outer_ids[oi]] = (int32_t)oi;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ void hset_insert(uint32_t* hs, uint32_t mask, uint32_t v, unsigned* err) {
    uint32_t h = hash32(v) & mask;
    for (uint32_t probes = 0; probes <= mask; ++probes) {
        uint32_t old = atomicCAS(&hs[h], 0xFFFFFFFFu, v);
        if (old == 0xFFFFFFFFu || old == v) return;
        h = (h + 1u) & mask;
    }
    atomicOr(err, ERR_HASH);
}

// One block per free row: the sorted column set (vertex ids) of the row.
// Count pass writes the numbers of free / constrained columns; fill pass
// writes all columns (vertex ids) at all_off and the split ff/fc columns.
// fill pass of a row: hs holds its U columns in its first n2 slots (n2 a
// power of two >= U, the rest EMPTY); sorted by a bitonic network, then
// written to the ff / fc rows with their ranks
__device__ __forceinline__ void row_pattern_fill(const RowPlan& rp, int64_t r, int U, int n2, uint32_t* hs,
                                                 const int64_t* ff_row_ptr, const int64_t* fc_row_ptr,
                                                 int32_t* all_cols, int32_t* ff_col, int32_t* fc_col) {
    const int t = threadIdx.x;
    __shared__ int csum[256];
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < n2; i += 256) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t a = hs[i], b = hs[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        hs[i] = b;
                        hs[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // fill: ranks among free / constrained columns by a block scan over chunks
    const int64_t ab = ff_row_ptr[r] + fc_row_ptr[r];
    int run_f = 0;
    for (int base = 0; base < U; base += 256) {
        const int i = base + t;
        const bool valid = i < U;
        const int32_t v = valid ? (int32_t)hs[i] : 0;
        const int32_t fid = valid ? rp.free_id[v] : -1;
        const int isf = (valid && fid >= 0) ? 1 : 0;
        csum[t] = isf;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int add = t >= off ? csum[t - off] : 0;
            __syncthreads();
            csum[t] += add;
            __syncthreads();
        }
        const int incl = csum[t];
        const int tot = csum[255];
        __syncthreads();
        if (valid) {
            all_cols[ab + i] = v;
            const int fr = run_f + incl - isf;  // free columns before i
            if (isf) ff_col[ff_row_ptr[r] + fr] = fid;
            else fc_col[fc_row_ptr[r] + (i - fr)] = v;
        }
        run_f += tot;
    }
}


// The count pass inserts the row's columns into an LDS hash set, counts them
// (free / constrained) and leaves them, unordered, in rowbuf (row r at
// r * row_stride; a row with more columns than row_stride sets ERR_ROWBUF and
// the host runs the pass again with a wider stride); the fill pass sorts them
// from there (LDS: row_stride words, a power of two) and writes the CSR rows.
template <bool FILL>
__global__ __launch_bounds__(256) void k_row_pattern(RowPlan rp, int hash_cap, int row_stride, int64_t* n_ff, int64_t* n_fc,
                                                     const int64_t* ff_row_ptr, const int64_t* fc_row_ptr,
                                                     int32_t* all_cols, int32_t* ff_col, int32_t* fc_col,
                                                     uint32_t* rowbuf, unsigned* err) {
    extern __shared__ uint32_t hs[];
    __shared__ int sU, sF;
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x;
    uint32_t* rb = rowbuf + r * (int64_t)row_stride;
    if constexpr (FILL) {
        // the row's columns as the count pass left them, padded to a power of
        // two with EMPTY for the sort
        const int U = (int)(n_ff[r] + n_fc[r]);
        int n2 = 1;
        while (n2 < U) n2 <<= 1;
        for (int i = t; i < n2; i += 256) hs[i] = i < U ? rb[i] : 0xFFFFFFFFu;
        __syncthreads();
        row_pattern_fill(rp, r, U, n2, hs, ff_row_ptr, fc_row_ptr, all_cols, ff_col, fc_col);
        return;
    }
    const int32_t u = rp.free_to_vertex[r];
    const uint32_t mask = (uint32_t)hash_cap - 1u;
    for (int i = t; i < hash_cap; i += 256) hs[i] = 0xFFFFFFFFu;
    if (t == 0) {
        sU = 0;
        sF = 0;
    }
    __syncthreads();
    // direct: ball vertex sets of outer tets containing u; inner-element
    // terms: vertices of T_Omega tets containing u that occur in some ball
    for (int64_t e4 = rp.vt_off[u]; e4 < rp.vt_off[u + 1]; ++e4) {
        const int64_t tl = rp.vt_val[e4];
        const int64_t e = tl >> 2;
        const int32_t oi = rp.outer_pos[e];
        if (oi >= 0)
            for (int64_t g = rp.ve_off[oi] + t; g < rp.ve_off[oi + 1]; g += 256)
                hset_insert(hs, mask, (uint32_t)rp.ve_ids[g], err);
        if (rp.region[e] && rp.inner_cnt[e] > 0 && t < 4) hset_insert(hs, mask, (uint32_t)rp.tets[4 * e + t], err);
    }
    // transposed: vertices of outer tets whose ball vertex set contains u
    for (int64_t k = rp.inc_off[u] + t; k < rp.inc_off[u + 1]; k += 256) {
        const int32_t oi = rp.ve_owner[rp.inc_val[k]];
        const int64_t n = rp.outer_ids[oi];
        for (int j = 0; j < 4; ++j) hset_insert(hs, mask, (uint32_t)rp.tets[4 * n + j], err);
    }
    __syncthreads();
    // the filled slots to rowbuf in any order (the fill pass sorts them), and
    // the free ones among them counted
    int nf = 0;
    for (int i = t; i < hash_cap; i += 256) {
        const uint32_t v = hs[i];
        if (v != 0xFFFFFFFFu) {
            const int q = atomicAdd(&sU, 1);
            if (q < row_stride) rb[q] = v;
            else atomicOr(err, ERR_ROWBUF);
            nf += rp.free_id[v] >= 0 ? 1 : 0;
        }
    }
    atomicAdd(&sF, nf);
    __syncthreads();
    if (t == 0) {
        n_ff[r] = sF;
        n_fc[r] = sU - sF;
    }
}
__device__ __forceinline__ int bsearch_cols(const int32_t* c, int n, int32_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Signed three-word fixed point for the row sums: |x| 2^s is split into an
// integer part and two 48-bit fraction words, each added (negated for x < 0)
// to its own 64-bit word.  Integer sums do not depend on the order of the
// terms, so a row is deterministic; a term is represented exactly unless it
// is below 2^-44 units of 2^-s, and then to 2^-96 units.  With at most 2^15
// terms per slot no word overflows.
constexpr unsigned long long kM48 = (1ull << 48) - 1ull;

__device__ __forceinline__ void fx3_add(unsigned long long* w, int stride, double x, double fx) {
    const double xs = fabs(x) * fx;
    const double h = floor(xs);
    const double r1 = (xs - h) * 281474976710656.0;  // exact: 48-bit shift of the fraction
    const double m = floor(r1);
    const double l = rint((r1 - m) * 281474976710656.0);
    unsigned long long H = (unsigned long long)h, Mi = (unsigned long long)m, Lo = (unsigned long long)l;
    if (x < 0.0) {
        H = 0ull - H;
        Mi = 0ull - Mi;
        Lo = 0ull - Lo;
    }
    atomicAdd(&w[0], H);
    atomicAdd(&w[stride], Mi);
    atomicAdd(&w[2 * stride], Lo);
}

// carry-normalised value: the magnitude words are made non-negative and
// below 2^48 before the (then exact) conversions, so tiny totals keep their
// relative precision
__device__ __forceinline__ double fx3_value(const unsigned long long* w, int stride, int shift) {
    long long h = (long long)w[0], m = (long long)w[stride], l = (long long)w[2 * stride];
    m += l >> 48;
    l &= (long long)kM48;
    h += m >> 48;
    m &= (long long)kM48;
    const bool neg = h < 0;
    if (neg) {
        l = -l;
        m = -m;
        h = -h;
        m += l >> 48;
        l &= (long long)kM48;
        h += m >> 48;
        m &= (long long)kM48;
    }
    const double v = ((double)l * 0x1p-96 + (double)m * 0x1p-48) + (double)h;
    const double r = ldexp(v, -shift);
    return neg ? -r : r;
}

// two-word value of the G accumulators (both words two's complement),
// carry-normalised before conversion: the fine word's carry by an arithmetic
// shift, its remainder in [0, 2^48)
__device__ __forceinline__ double fxs_value(unsigned long long hi, unsigned long long lo, int shift) {
    const long long h = (long long)hi + ((long long)lo >> 48);
    const double v = (double)(lo & kM48) * 0x1p-48 + (double)h;
    return ldexp(v, -shift);
}

// add x to the slot of column v (present in every row's pattern by construction)
__device__ __forceinline__ void slot_add(const int32_t* cols, int L, int32_t v, unsigned long long* acc, int stride,
                                         double x, double fx) {
    const int s = bsearch_cols(cols, L, v);
    if (s < L && cols[s] == v) fx3_add(acc + s, stride, x, fx);
}

__device__ __forceinline__ int tri4(int a, int b) {
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    const int rowstart[4] = {0, 4, 7, 9};
    return rowstart[a] + (b - a);
}

// G_m from its accumulators: the cut part (10 sums) plus the inside weight
// times the 4-point-rule moments of the whole tet (the inside case of the
// pair moments).
__global__ void k_g_finalize(int64_t K, const uint8_t* region, const int32_t* inner_cnt, const double* vol,
                             const unsigned long long* gacc, int g_shift, int w_shift, double* gvals) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K || !region[e] || inner_cnt[e] == 0) return;
    const unsigned long long* a = gacc + e;  // word i of tet e at a[i * K]
    const double win = fxs_value(a[20 * K], a[21 * K], w_shift);
    // S2 = sum_r (|E|/4) K_r K_r^T, K_r = barycentric coordinates of node r
    const double w = vol[e] * 0.25;
    double s2[10];
    for (int i = 0; i < 10; ++i) s2[i] = 0.0;
    for (int r = 0; r < 4; ++r) {
        int k = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = i; j < 4; ++j) {
                const double ki = (r == i) ? kAlpha : kBeta, kj = (r == j) ? kAlpha : kBeta;
                s2[k++] += (w * ki) * kj;
            }
    }
    for (int i = 0; i < 10; ++i)
        gvals[10 * e + i] = fxs_value(a[2 * i * K], a[(2 * i + 1) * K], g_shift) + win * s2[i];
}

// One block per free row.  GLOBAL: the row's three-word sums in global
// memory (racc, at 3 ab with stride L) and its columns read from all_cols,
// for rows too long for LDS; the same integers either way.
template <bool GLOBAL>
__global__ __launch_bounds__(256) void k_row_assemble(RowPlan rp, RowNumeric nm, unsigned long long* racc) {
    extern __shared__ unsigned long long sm[];
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x;
    const int32_t u = rp.free_to_vertex[r];
    const int64_t ab = rp.ff_row_ptr[r] + rp.fc_row_ptr[r];
    const int L = (int)(rp.ff_row_ptr[r + 1] + rp.fc_row_ptr[r + 1] - ab);
    const int st = GLOBAL ? L : rp.max_row;  // word stride of the accumulators
    unsigned long long* acc = GLOBAL ? racc + 3 * ab : sm;
    int32_t* cols_lds = (int32_t*)(sm + 3 * st);
    const int32_t* cols = GLOBAL ? rp.all_cols + ab : cols_lds;
    for (int i = t; i < L; i += 256) {
        if constexpr (!GLOBAL) cols_lds[i] = rp.all_cols[ab + i];
        acc[i] = 0ull;
        acc[st + i] = 0ull;
        acc[2 * st + i] = 0ull;
    }
    __syncthreads();
    const double fx = ldexp(1.0, nm.row_shift);
    // direct terms and the load vector of outer tets containing u
    for (int64_t e4 = rp.vt_off[u]; e4 < rp.vt_off[u + 1]; ++e4) {
        const int64_t tl = rp.vt_val[e4];
        const int64_t e = tl >> 2;
        const int j = (int)(tl & 3);
        const int32_t oi = rp.outer_pos[e];
        if (oi >= 0) {
            const int64_t vb = rp.ve_off[oi];
            const int U = (int)(rp.ve_off[oi + 1] - vb);
            const double* cb = nm.cblk + 4 * vb + j;
            for (int i = t; i < U; i += 256) slot_add(cols, L, rp.ve_ids[vb + i], acc, st, cb[4 * i], fx);
            if (t < 4) slot_add(cols, L, rp.tets[4 * e + t], acc, st, nm.oblk[20 * (int64_t)oi + 4 * j + t], fx);
        }
        if (rp.region[e] && rp.inner_cnt[e] > 0 && t < 4)
            slot_add(cols, L, rp.tets[4 * e + t], acc, st, nm.gvals[10 * e + tri4(j, t)], fx);
    }
    // transposed terms: entry g of the set Ve of outer tet oi holds u, so row
    // u receives C^oi[g][j] in the columns V_oi[j]
    for (int64_t k = rp.inc_off[u] + t; k < rp.inc_off[u + 1]; k += 256) {
        const int64_t g = rp.inc_val[k];
        const int32_t oi = rp.ve_owner[g];
        const int64_t n = rp.outer_ids[oi];
        const double4 cv = *(const double4*)(nm.cblk + 4 * g);
        const double c4[4] = {cv.x, cv.y, cv.z, cv.w};
        for (int jj = 0; jj < 4; ++jj) slot_add(cols, L, rp.tets[4 * n + jj], acc, st, c4[jj], fx);
    }
    __syncthreads();
    // values to the ff / fc blocks (columns are sorted; ranks by a block scan),
    // and per-thread partial sums of A_uv g_v over the constrained columns
    __shared__ int csum[256];
    __shared__ double red[256];
    double part = 0.0;
    int run_f = 0;
    for (int base = 0; base < L; base += 256) {
        const int i = base + t;
        const bool valid = i < L;
        const int32_t fid = valid ? rp.free_id[cols[i]] : -1;
        const int isf = (valid && fid >= 0) ? 1 : 0;
        csum[t] = isf;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int add = t >= off ? csum[t - off] : 0;
            __syncthreads();
            csum[t] += add;
            __syncthreads();
        }
        const int incl = csum[t];
        const int tot = csum[255];
        __syncthreads();
        if (valid) {
            const double val = fx3_value(acc + i, st, nm.row_shift);
            const int fr = run_f + incl - isf;
            if (isf) {
                nm.ff_val[rp.ff_row_ptr[r] + fr] = val;
            } else {
                nm.fc_val[rp.fc_row_ptr[r] + (i - fr)] = val;
                if (nm.g_nodal) part += val * nm.g_nodal[cols[i]];
            }
        }
        run_f += tot;
    }
    // b_u = sum over outer tets containing u of w c_u f  -  sum_fc A_uv g_v
    // (fixed-shape tree over the thread partials: deterministic)
    red[t] = part;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) {
        double f = 0.0;
        for (int64_t e4 = rp.vt_off[u]; e4 < rp.vt_off[u + 1]; ++e4) {
            const int64_t tl = rp.vt_val[e4];
            const int32_t oi = rp.outer_pos[tl >> 2];
            if (oi >= 0) f += nm.oblk[20 * (int64_t)oi + 16 + (tl & 3)];
        }
        nm.rhs[r] = f - red[0];
    }
}

}  // namespace

hipError_t launch_vt_keys(const int32_t* tets, int64_t K, uint64_t* keys, uint32_t* vals, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_vt_keys<<<blocks_for(4 * K), 256, 0, s>>>(tets, K, keys, vals);
    return hipGetLastError();
}

hipError_t launch_offsets(const uint64_t* skeys, int64_t n, int64_t n_keys, int64_t* off, hipStream_t s) {
    k_offsets<<<blocks_for(n + 1), 256, 0, s>>>(skeys, n, n_keys, off);
    return hipGetLastError();
}

hipError_t launch_inc_keys(const int64_t* ve_off, int64_t n_outer, const int32_t* ve_ids, uint64_t* keys,
                           uint32_t* vals, int32_t* owner, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_inc_keys<<<(unsigned)n_outer, 256, 0, s>>>(ve_off, n_outer, ve_ids, keys, vals, owner);
    return hipGetLastError();
}

hipError_t launch_inner_count(const int64_t* pair_off, int64_t n_outer, const int32_t* pair_m, int32_t* inner_cnt,
                              hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    const int64_t blocks = (n_outer + kInnerGroup - 1) / kInnerGroup;
    k_inner_count<<<(unsigned)blocks, 256, 0, s>>>(pair_off, n_outer, pair_m, inner_cnt);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<blocks_for(n), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_outer_pos(const int32_t* outer_ids, int64_t n_outer, int32_t* outer_pos, int64_t K, hipStream_t s) {
    if (K > 0) k_fill_i32<<<blocks_for(K), 256, 0, s>>>(outer_pos, K, -1);
    if (n_outer > 0) k_outer_pos<<<blocks_for(n_outer), 256, 0, s>>>(outer_ids, n_outer, outer_pos);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<blocks_for(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_row_pattern(bool fill, const RowPlan& rp, int64_t n_rows, int hash_cap, int row_stride, int64_t* n_ff,
                              int64_t* n_fc, const int64_t* ff_row_ptr, const int64_t* fc_row_ptr, int32_t* all_cols,
                              int32_t* ff_col, int32_t* fc_col, uint32_t* rowbuf, unsigned* err, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    // the stride must be a power of two no larger than the hash set (the fill
    // pass sorts a row in row_stride words of LDS)
    if (row_stride <= 0 || row_stride > hash_cap || (row_stride & (row_stride - 1)) != 0) return hipErrorInvalidValue;
    if (fill)
        k_row_pattern<true><<<(unsigned)n_rows, 256, (size_t)row_stride * 4, s>>>(
            rp, hash_cap, row_stride, n_ff, n_fc, ff_row_ptr, fc_row_ptr, all_cols, ff_col, fc_col, rowbuf, err);
    else
        k_row_pattern<false><<<(unsigned)n_rows, 256, (size_t)hash_cap * 4, s>>>(
            rp, hash_cap, row_stride, n_ff, n_fc, ff_row_ptr, fc_row_ptr, all_cols, ff_col, fc_col, rowbuf, err);
    return hipGetLastError();
}

hipError_t launch_g_finalize(int64_t K, const uint8_t* region, const int32_t* inner_cnt, const double* vol,
                             const unsigned long long* gacc, int g_shift, int w_shift, double* gvals, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_g_finalize<<<blocks_for(K), 256, 0, s>>>(K, region, inner_cnt, vol, gacc, g_shift, w_shift, gvals);
    return hipGetLastError();
}

size_t row_assemble_lds_bytes(int max_row) { return (size_t)max_row * 28 + 64; }
size_t row_assemble_static_lds() { return 256 * (sizeof(int) + sizeof(double)) + 64; }

hipError_t launch_row_assemble(const RowPlan& rp, const RowNumeric& nm, int64_t n_rows, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    k_row_assemble<false><<<(unsigned)n_rows, 256, row_assemble_lds_bytes(rp.max_row), s>>>(rp, nm, nullptr);
    return hipGetLastError();
}

hipError_t launch_row_assemble_global(const RowPlan& rp, const RowNumeric& nm, unsigned long long* racc,
                                      int64_t n_rows, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    k_row_assemble<true><<<(unsigned)n_rows, 256, 0, s>>>(rp, nm, racc);
    return hipGetLastError();
}

}  // namespace nlfem
