// Symbolic phase: device mesh layout, uniform-grid cell list, exact FP64
// ball classification of every (outer point, tet) pair, local vertex sets of
// each outer tet.  The CSR pattern is built row by row in k_rows.hip.
#include "device_geom.hpp"

namespace nlfem {

namespace {

__device__ __forceinline__ unsigned long long ordered_bits(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// per tet: validate indices, gather coordinates (row-major [4][3]), volume
// |det|/6, region, bounding-box minimum corner; global max extent and bbox.
__global__ __launch_bounds__(256) void k_mesh_prep(MeshDev m, double* tetX, double* vol, uint8_t* region,
                                                   double* tet_min, unsigned long long* ext_bits,
                                                   unsigned long long* bbox_bits, unsigned* err) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.K) return;
    int32_t v[4];
    bool ok = true;
    for (int l = 0; l < 4; ++l) {
        v[l] = m.tets[4 * e + l];
        ok = ok && v[l] >= 0 && (int64_t)v[l] < m.V;
    }
    if (!ok) {
        atomicOr(err, ERR_INDEX);
        for (int i = 0; i < 12; ++i) tetX[12 * e + i] = 0.0;
        vol[e] = 0.0;
        region[e] = 0;
        for (int i = 0; i < 3; ++i) tet_min[3 * e + i] = 0.0;
        return;
    }
    double X[12];
    for (int l = 0; l < 4; ++l)
        for (int i = 0; i < 3; ++i) X[3 * l + i] = m.coords[3 * (int64_t)v[l] + i];
    for (int i = 0; i < 12; ++i) tetX[12 * e + i] = X[i];
    double V6 = fabs(orient3(X, X + 3, X + 6, X + 9)) / 6.0;
    vol[e] = V6;
    if (!(V6 > 0.0)) atomicOr(err, ERR_VOLUME);
    bool anyfree = false;
    for (int l = 0; l < 4; ++l) anyfree = anyfree || (m.vfree[v[l]] != 0);
    uint8_t rg = m.region_in ? (m.region_in[e] ? 1 : 0) : (anyfree ? 1 : 0);
    if (!rg && anyfree) atomicOr(err, ERR_REGION);
    region[e] = rg;
    double ext = 0.0;
    for (int i = 0; i < 3; ++i) {
        double lo = fmin(fmin(X[i], X[3 + i]), fmin(X[6 + i], X[9 + i]));
        double hi = fmax(fmax(X[i], X[3 + i]), fmax(X[6 + i], X[9 + i]));
        tet_min[3 * e + i] = lo;
        ext = fmax(ext, hi - lo);
        atomicMin(&bbox_bits[i], ordered_bits(lo));
        atomicMax(&bbox_bits[3 + i], ordered_bits(hi));
    }
    atomicMax(ext_bits, ordered_bits(ext));
}

__global__ void k_init_bits(unsigned long long* ext_bits, unsigned long long* bbox_bits) {
    *ext_bits = 0ull;
    for (int i = 0; i < 3; ++i) {
        bbox_bits[i] = ~0ull;
        bbox_bits[3 + i] = 0ull;
    }
}

__global__ void k_decode_bits(const unsigned long long* bits, int n, double* out) {
    int i = threadIdx.x;
    if (i < n) {
        unsigned long long b = bits[i];
        unsigned long long r = (b >> 63) ? (b & 0x7FFFFFFFFFFFFFFFull) : ~b;
        out[i] = __longlong_as_double((long long)r);
    }
}

__global__ void k_free_ids(const uint8_t* vfree, const int32_t* scan, int64_t V, int32_t* free_id,
                           int32_t* free_to_vertex) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    if (vfree[v]) {
        free_id[v] = scan[v];
        free_to_vertex[scan[v]] = (int32_t)v;
    } else {
        free_id[v] = -1;
    }
}

__global__ void k_outer_flags(const uint8_t* region, const uint8_t* mask, int64_t K, int64_t* flags) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    flags[e] = (region[e] && (!mask || mask[e])) ? 1 : 0;
}

__global__ void k_outer_compact(const int64_t* flags, const int64_t* scan, int64_t K, int32_t* outer_ids) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    if (flags[e]) outer_ids[scan[e]] = (int32_t)e;
}

__device__ __forceinline__ int cell_coord(double x, double o, double cs, int n) {
    double f = floor((x - o) / cs);
    if (f < 0.0) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int)f;
}

__global__ void k_cell_keys(const double* tet_min, int64_t K, Grid g, uint64_t* keys, uint32_t* vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    int cx = cell_coord(tet_min[3 * e], g.ox, g.cs, g.nx);
    int cy = cell_coord(tet_min[3 * e + 1], g.oy, g.cs, g.ny);
    int cz = cell_coord(tet_min[3 * e + 2], g.oz, g.cs, g.nz);
    keys[e] = (uint64_t)cx + (uint64_t)g.nx * ((uint64_t)cy + (uint64_t)g.ny * (uint64_t)cz);
    vals[e] = (uint32_t)e;
}

// cell_start[c] = first sorted position with key >= c; cell_start[n_cells] = K
__global__ void k_cell_start(const uint64_t* skeys, int64_t K, int64_t n_cells, int64_t* cell_start) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > K) return;
    int64_t prev = (i == 0) ? -1 : (int64_t)skeys[i - 1];
    int64_t cur = (i == K) ? n_cells : (int64_t)skeys[i];
    for (int64_t c = prev + 1; c <= cur; ++c) cell_start[c] = i;
}

// Candidate cells of one outer tet.  Every tet that meets one of the four
// balls B(p_k, delta) has a point y with |y - c| < R (c = mean of the p_k,
// R = delta + max_k |p_k - c|, inflated by 1e-7), and its bounding-box minimum
// corner t lies within one cell side below y on every axis.  A cell row
// (cy, cz) is visited only if the slab of possible y over that row comes
// closer than R to c, and then only over the x cells that can hold t.  Cell
// boundaries are widened by 1e-6 cells and one guard cell on each end of a
// range absorbs rounding of the cell index, so the candidate set contains
// every tet that the exact test can find.
struct CandBall {
    double c[3];
    double R;
};

__device__ __forceinline__ CandBall cand_ball(const double P[4][3], double delta) {
    CandBall b;
    for (int i = 0; i < 3; ++i) b.c[i] = 0.25 * ((P[0][i] + P[1][i]) + (P[2][i] + P[3][i]));
    double r = 0.0;
    for (int k = 0; k < 4; ++k) {
        double dx = P[k][0] - b.c[0], dy = P[k][1] - b.c[1], dz = P[k][2] - b.c[2];
        r = fmax(r, sqrt((dx * dx + dy * dy) + dz * dz));
    }
    b.R = (delta + r) * (1.0 + 1e-7);
    return b;
}

__device__ __forceinline__ int clampi(double v, int n) { return v < 0.0 ? 0 : (v > (double)(n - 1) ? n - 1 : (int)v); }

__device__ __forceinline__ double slab_gap(double c, double o, double cs, int cidx) {
    const double m = 1e-6 * cs;
    const double lo = o + (double)cidx * cs - m, hi = o + (double)(cidx + 2) * cs + m;
    return fmax(fmax(lo - c, c - hi), 0.0);
}

// range of cell rows along one axis
__device__ __forceinline__ void axis_range(const CandBall& b, int ax, const Grid& g, int& lo, int& hi) {
    const double o = ax == 0 ? g.ox : (ax == 1 ? g.oy : g.oz);
    const int n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
    lo = clampi(floor((b.c[ax] - b.R - g.cs - o) / g.cs) - 1.0, n);
    hi = clampi(floor((b.c[ax] + b.R - o) / g.cs) + 1.0, n);
}

// x cells of row (cy, cz); returns false if the row is skipped
__device__ __forceinline__ bool row_range(const CandBall& b, const Grid& g, int cy, int cz, int& x0, int& x1) {
    const double dy = slab_gap(b.c[1], g.oy, g.cs, cy);
    const double dz = slab_gap(b.c[2], g.oz, g.cs, cz);
    const double rem = b.R * b.R - (dy * dy + dz * dz);
    if (!(rem > 0.0)) return false;
    const double hw = sqrt(rem);
    x0 = clampi(floor((b.c[0] - hw - g.cs - g.ox) / g.cs) - 1.0, g.nx);
    x1 = clampi(floor((b.c[0] + hw - g.ox) / g.cs) + 1.0, g.nx);
    return true;
}

__device__ __forceinline__ void load_outer_points(const double* tetX, int n, double P[4][3]) {
    double Xn[12];
    for (int i = 0; i < 12; ++i) Xn[i] = tetX[12 * (int64_t)n + i];
    for (int k = 0; k < 4; ++k) outer_point(Xn, k, P[k]);
}

// candidates per outer tet (an upper bound of its pair count)
__global__ void k_cand_count(const double* tetX, const int32_t* outer_ids, int64_t n_outer, const int64_t* cell_start,
                             Grid g, double delta, int64_t* cand) {
    const int64_t oi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (oi >= n_outer) return;
    double P[4][3];
    load_outer_points(tetX, outer_ids[oi], P);
    const CandBall b = cand_ball(P, delta);
    int y0, y1, z0, z1;
    axis_range(b, 1, g, y0, y1);
    axis_range(b, 2, g, z0, z1);
    int64_t tot = 0;
    for (int cz = z0; cz <= z1; ++cz)
        for (int cy = y0; cy <= y1; ++cy) {
            int x0, x1;
            if (!row_range(b, g, cy, cz, x0, x1)) continue;
            const int64_t row = (int64_t)g.nx * ((int64_t)cy + (int64_t)g.ny * cz);
            tot += cell_start[row + x1 + 1] - cell_start[row + x0];
        }
    cand[oi] = tot;
}

// One wave per outer tet: exact classification of every candidate for the
// four outer points; hits go to the tet's candidate region in candidate
// order, with their count per "number of cut points" bucket.
__global__ __launch_bounds__(256) void k_classify(const double* tetX, const int32_t* outer_ids, int64_t n_outer,
                                                  const int64_t* cell_start, const uint32_t* cell_tets, Grid g,
                                                  double delta, const int64_t* cand_off, int64_t* cnt, int32_t* hit_m,
                                                  uint16_t* hit_cls) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    double P[4][3];
    load_outer_points(tetX, outer_ids[oi], P);
    const double d2 = delta * delta;
    const CandBall b = cand_ball(P, delta);
    int y0, y1, z0, z1;
    axis_range(b, 1, g, y0, y1);
    axis_range(b, 2, g, z0, z1);
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = cand_off[oi];
    int64_t nhit = 0;
    int64_t c[5] = {0, 0, 0, 0, 0};
    for (int cz = z0; cz <= z1; ++cz) {
        for (int cy = y0; cy <= y1; ++cy) {
            int x0, x1;
            if (!row_range(b, g, cy, cz, x0, x1)) continue;
            const int64_t row = (int64_t)g.nx * ((int64_t)cy + (int64_t)g.ny * cz);
            const int64_t beg = cell_start[row + x0], end = cell_start[row + x1 + 1];
            for (int64_t j = beg; j < end; j += 64) {
                const int64_t idx = j + lane;
                const bool valid = idx < end;
                uint32_t code = 0;
                int ncut = 0;
                bool hit = false;
                int m = 0;
                if (valid) {
                    m = (int)cell_tets[idx];
                    double X[12];
                    for (int i = 0; i < 12; ++i) X[i] = tetX[12 * (int64_t)m + i];
                    for (int k = 0; k < 4; ++k) {
                        double r2[4];
                        const int cl = classify(X, P[k], d2, r2);
                        code |= (uint32_t)cl << (3 * k);
                        hit = hit || (cl != C_OUT);
                        ncut += (cl >= C_CUT0) ? 1 : 0;
                    }
                }
                const uint64_t mask = __ballot(hit);
                if (hit) {
                    const int64_t pos = base + nhit + __popcll(mask & lt);
                    hit_m[pos] = m;
                    hit_cls[pos] = (uint16_t)(code | ((uint32_t)ncut << 12));
                }
                nhit += __popcll(mask);
                for (int bb = 0; bb <= 4; ++bb) c[bb] += __popcll(__ballot(hit && ncut == bb));
            }
        }
    }
    if (lane == 0)
        for (int bb = 0; bb < 5; ++bb) cnt[oi * 5 + bb] = c[bb];
}

// which of the 4 outer points cut the tet (bit k set: class of point k is CUT)
__device__ __forceinline__ int cut_mask(uint32_t code) {
    int mk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mk |= ((((code >> (3 * k)) & 7u) >= (uint32_t)C_CUT0) ? 1 : 0) << k;
    return mk;
}

// One wave per outer tet: the hits, grouped by their cut mask (more cut
// points first, then the larger mask) and in candidate order within a group,
// to the final pair arrays.  Lanes of a wave then see the same cut points, so
// the sample loops of a wave are not run for points that only some lanes cut.
__global__ __launch_bounds__(256) void k_pair_compact(int64_t n_outer, const int64_t* cand_off, const int64_t* cnt,
                                                      const int64_t* pair_off, const int32_t* hit_m,
                                                      const uint16_t* hit_cls, int32_t* pair_m, uint16_t* pair_cls) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    (void)cnt;
    const int64_t n = pair_off[oi + 1] - pair_off[oi];
    const int64_t src = cand_off[oi];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t c[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    for (int64_t j = 0; j < n; j += 64) {
        const bool valid = j + lane < n;
        const int mk = valid ? cut_mask(hit_cls[src + j + lane]) : -1;
#pragma unroll
        for (int b = 0; b < 16; ++b) c[b] += __popcll(__ballot(mk == b));
    }
    // group order: 15 | 14 13 11 7 | 12 10 9 6 5 3 | 8 4 2 1 | 0
    const int order[16] = {15, 14, 13, 11, 7, 12, 10, 9, 6, 5, 3, 8, 4, 2, 1, 0};
    int64_t base[16];
    int64_t run = pair_off[oi];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        base[order[i]] = run;
        run += c[order[i]];
    }
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    for (int64_t j = 0; j < n; j += 64) {
        const bool valid = j + lane < n;
        const uint32_t code = valid ? hit_cls[src + j + lane] : 0u;
        const int m = valid ? hit_m[src + j + lane] : 0;
        const int mk = valid ? cut_mask(code) : -1;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const bool mine = mk == b;
            const uint64_t mask = __ballot(mine);
            if (mine) {
                const int64_t pos = base[b] + c[b] + __popcll(mask & lt);
                pair_m[pos] = m;
                pair_cls[pos] = (uint16_t)(code & 0xFFFu);
            }
            c[b] += __popcll(mask);
        }
    }
}

__global__ void k_pair_totals(const int64_t* cnt, int64_t n_outer, int64_t* tot) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_outer) return;
    tot[i] = cnt[5 * i] + cnt[5 * i + 1] + cnt[5 * i + 2] + cnt[5 * i + 3] + cnt[5 * i + 4];
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// One block per outer tet: the sorted set Ve of vertices of the inner tets of
// its pair list (LDS hash set, then bitonic sort).  The count pass writes |Ve|,
// the fill pass the set itself at ve_off.
template <bool FILL>
__global__ __launch_bounds__(256) void k_pattern(const int32_t* tets, int64_t n_outer, const int64_t* pair_off,
                                                 const int32_t* pair_m, int hash_cap, int64_t* ucount,
                                                 const int64_t* ve_off, int32_t* ve_ids, unsigned* err) {
    extern __shared__ uint32_t hs[];
    __shared__ int sU;
    const uint32_t EMPTY = 0xFFFFFFFFu;
    const int64_t oi = blockIdx.x;
    const int t = threadIdx.x;
    for (int i = t; i < hash_cap; i += 256) hs[i] = EMPTY;
    if (t == 0) sU = 0;
    __syncthreads();
    const int64_t p0 = pair_off[oi], p1 = pair_off[oi + 1];
    const uint32_t hmask = (uint32_t)hash_cap - 1u;
    for (int64_t p = p0 + t; p < p1; p += 256) {
        int m = pair_m[p];
        for (int j = 0; j < 4; ++j) {
            uint32_t v = (uint32_t)tets[4 * (int64_t)m + j];
            uint32_t h = hash32(v) & hmask;
            int probes = 0;
            while (true) {
                uint32_t old = atomicCAS(&hs[h], EMPTY, v);
                if (old == EMPTY || old == v) break;
                h = (h + 1u) & hmask;
                if (++probes >= hash_cap) {
                    atomicOr(err, ERR_HASH);
                    break;
                }
            }
        }
    }
    __syncthreads();
    for (int k = 2; k <= hash_cap; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < hash_cap; i += 256) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint32_t a = hs[i], b = hs[ixj];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        hs[i] = b;
                        hs[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = t; i < hash_cap; i += 256)
        if (hs[i] != EMPTY && (i == hash_cap - 1 || hs[i + 1] == EMPTY)) sU = i + 1;
    __syncthreads();
    const int U = sU;
    if (!FILL) {
        if (t == 0) ucount[oi] = U;
        return;
    }
    const int64_t vb = ve_off[oi];
    for (int i = t; i < U; i += 256) ve_ids[vb + i] = (int32_t)hs[i];
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_mesh_prep(const MeshDev& m, double* tetX, double* vol, uint8_t* region, double* tet_min,
                            double* ext_max_dev, double* bbox_dev, unsigned* err, hipStream_t s) {
    // ext_max_dev / bbox_dev: 7 doubles of output; bits scratch placed after them
    unsigned long long* bits = (unsigned long long*)(bbox_dev + 6);
    k_init_bits<<<1, 1, 0, s>>>(bits, bits + 1);
    if (m.K > 0)
        k_mesh_prep<<<blocks_for(m.K), 256, 0, s>>>(m, tetX, vol, region, tet_min, bits, bits + 1, err);
    k_decode_bits<<<1, 64, 0, s>>>(bits, 1, ext_max_dev);
    k_decode_bits<<<1, 64, 0, s>>>(bits + 1, 6, bbox_dev);
    return hipGetLastError();
}

hipError_t launch_free_ids(const uint8_t* vfree, const int32_t* scan, int64_t V, int32_t* free_id,
                           int32_t* free_to_vertex, hipStream_t s) {
    if (V <= 0) return hipSuccess;
    k_free_ids<<<blocks_for(V), 256, 0, s>>>(vfree, scan, V, free_id, free_to_vertex);
    return hipGetLastError();
}

hipError_t launch_outer_flags(const uint8_t* region, const uint8_t* mask, int64_t K, int64_t* flags, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_outer_flags<<<blocks_for(K), 256, 0, s>>>(region, mask, K, flags);
    return hipGetLastError();
}

hipError_t launch_outer_compact(const int64_t* flags, const int64_t* scan, int64_t K, int32_t* outer_ids,
                                hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_outer_compact<<<blocks_for(K), 256, 0, s>>>(flags, scan, K, outer_ids);
    return hipGetLastError();
}

hipError_t launch_cell_keys(const double* tet_min, int64_t K, Grid g, uint64_t* keys, uint32_t* vals,
                            hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_cell_keys<<<blocks_for(K), 256, 0, s>>>(tet_min, K, g, keys, vals);
    return hipGetLastError();
}

hipError_t launch_cell_start(const uint64_t* sorted_keys, int64_t K, int64_t n_cells, int64_t* cell_start,
                             hipStream_t s) {
    k_cell_start<<<blocks_for(K + 1), 256, 0, s>>>(sorted_keys, K, n_cells, cell_start);
    return hipGetLastError();
}

hipError_t launch_cand_count(const double* tetX, const int32_t* outer_ids, int64_t n_outer,
                             const int64_t* cell_start, Grid g, double delta, int64_t* cand, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_cand_count<<<blocks_for(n_outer), 256, 0, s>>>(tetX, outer_ids, n_outer, cell_start, g, delta, cand);
    return hipGetLastError();
}

hipError_t launch_classify(const double* tetX, const int32_t* outer_ids, int64_t n_outer, const int64_t* cell_start,
                           const uint32_t* cell_tets, Grid g, double delta, const int64_t* cand_off, int64_t* cnt,
                           int32_t* hit_m, uint16_t* hit_cls, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_classify<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(tetX, outer_ids, n_outer, cell_start, cell_tets, g, delta,
                                                             cand_off, cnt, hit_m, hit_cls);
    return hipGetLastError();
}

hipError_t launch_pair_compact(int64_t n_outer, const int64_t* cand_off, const int64_t* cnt, const int64_t* pair_off,
                               const int32_t* hit_m, const uint16_t* hit_cls, int32_t* pair_m, uint16_t* pair_cls,
                               hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_pair_compact<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(n_outer, cand_off, cnt, pair_off, hit_m, hit_cls,
                                                                 pair_m, pair_cls);
    return hipGetLastError();
}

hipError_t launch_pair_totals(const int64_t* cnt, int64_t n_outer, int64_t* tot, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_pair_totals<<<blocks_for(n_outer), 256, 0, s>>>(cnt, n_outer, tot);
    return hipGetLastError();
}

hipError_t launch_pattern(bool fill, const int32_t* tets, int64_t n_outer, const int64_t* pair_off,
                          const int32_t* pair_m, int hash_cap, int64_t* ucount, const int64_t* ve_off, int32_t* ve_ids,
                          unsigned* err, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    size_t sh = (size_t)hash_cap * sizeof(uint32_t);
    if (fill)
        k_pattern<true><<<(unsigned)n_outer, 256, sh, s>>>(tets, n_outer, pair_off, pair_m, hash_cap, ucount, ve_off,
                                                          ve_ids, err);
    else
        k_pattern<false><<<(unsigned)n_outer, 256, sh, s>>>(tets, n_outer, pair_off, pair_m, hash_cap, ucount,
                                                           ve_off, ve_ids, err);
    return hipGetLastError();
}

}  // namespace nlfem
