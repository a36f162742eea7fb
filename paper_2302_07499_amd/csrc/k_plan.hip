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
// |det|/6, region, bounding-box minimum corner; global max extent and bbox
// (reduced over each wave first: one set of device-wide atomics per wave
// instead of per tet, which all hit the same seven words).
__global__ __launch_bounds__(256) void k_mesh_prep(MeshDev m, double* tetX, double* vol, uint8_t* region,
                                                   double* tet_min, unsigned long long* ext_bits,
                                                   unsigned long long* bbox_bits, unsigned* err) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // ordered bits of the tet's box and extent; the identities for lanes without a valid tet
    unsigned long long lo_b[3] = {~0ull, ~0ull, ~0ull}, hi_b[3] = {0ull, 0ull, 0ull}, ext_b = 0ull;
    if (e < m.K) {
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
        } else {
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
                lo_b[i] = ordered_bits(lo);
                hi_b[i] = ordered_bits(hi);
            }
            ext_b = ordered_bits(ext);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const unsigned long long ol = __shfl_xor(lo_b[i], off, 64), oh = __shfl_xor(hi_b[i], off, 64);
            lo_b[i] = ol < lo_b[i] ? ol : lo_b[i];
            hi_b[i] = oh > hi_b[i] ? oh : hi_b[i];
        }
        const unsigned long long ox = __shfl_xor(ext_b, off, 64);
        ext_b = ox > ext_b ? ox : ext_b;
    }
    if ((threadIdx.x & 63) == 0 && ext_b != 0ull) {
        for (int i = 0; i < 3; ++i) {
            atomicMin(&bbox_bits[i], lo_b[i]);
            atomicMax(&bbox_bits[3 + i], hi_b[i]);
        }
        atomicMax(ext_bits, ext_b);
    }
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
// boundaries and the x ranges are widened by 1e-6 cells (the rounding of a
// cell index, on either side, is below 1e-8 cells: a few roundings of at most
// 2^-53 of a value below 2^24 cells; R carries 1e-7 relative for the rounding
// of the chord) and the row ranges by one guard row, so the candidate set
// contains every tet that the exact test can find.
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
    x0 = clampi(floor((b.c[0] - hw - g.cs - g.ox) / g.cs - 1e-6), g.nx);
    x1 = clampi(floor((b.c[0] + hw - g.ox) / g.cs + 1e-6), g.nx);
    return true;
}

__device__ __forceinline__ void load_outer_points(const double* tetX, int n, double P[4][3]) {
    double Xn[12];
    for (int i = 0; i < 12; ++i) Xn[i] = tetX[12 * (int64_t)n + i];
    for (int k = 0; k < 4; ++k) outer_point(Xn, k, P[k]);
}

// Bounding boxes of the tets in cell order (box[2j], box[2j+1] = lower and
// upper corner of tet cell_tets[j]), in float rounded outward, so that the
// classification can drop far candidates with one coalesced 32-byte read;
// and the tets' vertex blocks in the same order (sX[j] = tetX[cell_tets[j]]),
// so that the candidates it keeps read theirs coalesced, without first
// loading the tet id.
__global__ void k_sorted_boxes(const double* tetX, const uint32_t* cell_tets, int64_t K, float4* box, double* sX) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const double* X = tetX + 12 * (int64_t)cell_tets[j];
    float lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        lo[i] = __double2float_rd(fmin(fmin(X[i], X[3 + i]), fmin(X[6 + i], X[9 + i])));
        hi[i] = __double2float_ru(fmax(fmax(X[i], X[3 + i]), fmax(X[6 + i], X[9 + i])));
    }
    box[2 * j] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    box[2 * j + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    for (int i = 0; i < 12; ++i) sX[12 * j + i] = X[i];
}

// squared distance from p to a box, computed in double from the (outward
// rounded) float corners: never above the distance to the tet's own box
__device__ __forceinline__ double box_dist2(const float4& lo, const float4& hi, const double* p) {
    const double gx = fmax(fmax((double)lo.x - p[0], p[0] - (double)hi.x), 0.0);
    const double gy = fmax(fmax((double)lo.y - p[1], p[1] - (double)hi.y), 0.0);
    const double gz = fmax(fmax((double)lo.z - p[2], p[2] - (double)hi.z), 0.0);
    return (gx * gx + gy * gy) + gz * gz;
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

// Classification in three passes over the candidate regions of the outer
// tets (region of outer tet oi: [cand_off[oi], cand_off[oi+1]), candidates
// in (cell row, cell, cell list) order):
//   k_classify_fast   one wave per outer tet drops candidates whose (sorted,
//                     float) bounding box is beyond delta of all four points,
//                     classifies the rest (one class byte per outer point:
//                     IN / CUT(n_in) / OUT, or kPending when only the exact
//                     closed-tet test can decide between CUT(0) and OUT) and
//                     writes those not OUT for every point compacted at the
//                     start of the region (count in cand_n);
//   k_classify_exact  one block per outer tet queues the pending (candidate,
//                     point) cases in LDS and tests them densely, patches the
//                     codes, and counts the hits per "number of cut points";
//   k_pair_compact    (below) gathers the hits into the pair arrays.
constexpr uint32_t kPending = 0xFFu;

// orders this wave's LDS writes before its later reads (a wave runs in
// lockstep; the fences keep the compiler from reordering across)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// classes of the near candidate j against the four points (one byte per
// point: IN, CUT(n_in), kPending, or 0 = OUT)
__device__ __forceinline__ uint32_t classify_candidate(const double* sX, int64_t j, const double (*P)[3], double d2,
                                                       int strategy) {
    double X[12];
    {
        const double2* xs = (const double2*)(sX + 12 * j);  // 96-byte rows: 16-byte aligned
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const double2 v = xs[i];
            X[2 * i] = v.x;
            X[2 * i + 1] = v.y;
        }
    }
    uint32_t code = 0;
    for (int k = 0; k < 4; ++k) {
        int cl;
        if (strategy == S_BARYCENTER) {
            cl = barycenter_inside(X, P[k], d2) ? C_IN : C_OUT;
        } else {
            cl = classify_fast(X, P[k], d2);
            // inside: only whole-inside elements; nothing is left pending
            if (strategy == S_INSIDE && cl != C_IN) cl = C_OUT;
        }
        code |= (cl < 0 ? kPending : (uint32_t)cl) << (8 * k);
    }
    return code;
}

// cell rows of one outer tet's candidate region kept in LDS (up to kMaxRows
// at a time), so that the wave walks the region as one list in full 64-lane
// chunks across rows; the candidates whose box passes the ball test are
// queued (kNearQ slots per wave) and classified in full rounds of 64
constexpr int kMaxRows = 256;
constexpr int kNearQ = 128;  // < 64 left over + 64 appended per chunk

__global__ __launch_bounds__(256) void k_classify_fast(const double* tetX, const int32_t* outer_ids, int64_t n_outer,
                                                       const int64_t* cell_start, const uint32_t* cell_tets,
                                                       const float4* box, const double* sX, Grid g, double delta,
                                                       int strategy,
                                                       const int64_t* cand_off, int64_t* cand_n, int32_t* cand_m,
                                                       uint32_t* cand_code) {
    __shared__ int64_t row_beg[4][kMaxRows];
    __shared__ int64_t row_pre[4][kMaxRows + 1];  // candidates before each row
    __shared__ int64_t near_q[4][kNearQ];         // queued near candidates (cell order)
    // the wave index is uniform: in a scalar register, the outer tet and its points are too
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    double P[4][3];
    load_outer_points(tetX, outer_ids[oi], P);
    const double d2 = delta * delta;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    // the ball around the points' centre that holds their four balls (radius
    // delta + the largest distance to a point, enlarged by 1e-7): a box beyond
    // it is beyond delta of every point, so one box test per candidate drops
    // the far ones and the classes are unchanged
    const CandBall b = cand_ball(P, delta);
    const double bR2 = b.R * b.R;
    int y0, y1, z0, z1;
    axis_range(b, 1, g, y0, y1);
    axis_range(b, 2, g, z0, z1);
    // the candidates with a class other than OUT for some point are written
    // compacted, in candidate order, from the start of the region
    const int64_t base = cand_off[oi];
    int64_t n_hit = 0;
    auto emit = [&](uint32_t code, int m) {
        const bool hit = code != 0u;
        const uint64_t bal = __ballot(hit);
        if (hit) {
            const int64_t pos = base + n_hit + __popcll(bal & lt);
            cand_m[pos] = m;
            cand_code[pos] = code;
        }
        n_hit += __popcll(bal);
    };
    // classify queue entry `lane` when it is below n (all lanes take part in emit)
    int64_t* Q = near_q[wave];
    auto classify_round = [&](int n) {
        uint32_t code = 0;
        int m = 0;
        if (lane < n) {
            const int64_t j = Q[lane];
            m = (int)cell_tets[j];
            code = classify_candidate(sX, j, P, d2, strategy);
        }
        emit(code, m);
    };
    int nq = 0;
    const int ny = y1 - y0 + 1;
    const int n_rows = (z1 >= z0 && y1 >= y0) ? ny * (z1 - z0 + 1) : 0;
    int64_t* RB = row_beg[wave];
    int64_t* RP = row_pre[wave];
    // rows in (cz, cy) order, kMaxRows at a time: their first candidate and a
    // running count, then the candidates of those rows as one list
    for (int rb = 0; rb < n_rows; rb += kMaxRows) {
        const int nr = min(kMaxRows, n_rows - rb);
        int64_t run = 0;
        for (int r0 = 0; r0 < nr; r0 += 64) {
            const int r = r0 + lane;
            int64_t cnt = 0, beg = 0;
            if (r < nr) {
                const int cz = z0 + (rb + r) / ny, cy = y0 + (rb + r) % ny;
                int x0, x1;
                if (row_range(b, g, cy, cz, x0, x1)) {
                    const int64_t row = (int64_t)g.nx * ((int64_t)cy + (int64_t)g.ny * cz);
                    beg = cell_start[row + x0];
                    cnt = cell_start[row + x1 + 1] - beg;
                }
            }
            // inclusive scan of the counts across the wave
            int64_t inc = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const int64_t v = __shfl_up(inc, off, 64);
                if (lane >= off) inc += v;
            }
            if (r < nr) {
                RB[r] = beg;
                RP[r] = run + inc - cnt;
            }
            run += __shfl(inc, 63, 64);
        }
        if (lane == 0) RP[nr] = run;
        wave_sync();
        int r = 0;  // this lane's row cursor: its candidate index only grows
        for (int64_t c0 = 0; c0 < run; c0 += 64) {
            const int64_t c = c0 + lane;
            bool near = false;
            int64_t j = 0;
            if (c < run) {
                while (RP[r + 1] <= c) ++r;
                j = RB[r] + (c - RP[r]);
                near = !(box_dist2(box[2 * j], box[2 * j + 1], b.c) > bR2);
            }
            const uint64_t bal = __ballot(near);
            if (near) Q[nq + __popcll(bal & lt)] = j;
            nq += __popcll(bal);
            wave_sync();
            if (nq >= 64) {
                classify_round(64);
                // move the rest of the queue (fewer than 64) down
                const int rest = nq - 64;
                const int64_t keep = lane < rest ? Q[64 + lane] : 0;
                wave_sync();
                if (lane < rest) Q[lane] = keep;
                wave_sync();
                nq = rest;
            }
        }
        wave_sync();  // the next batch of rows overwrites RB and RP
    }
    if (nq > 0) classify_round(nq);
    if (lane == 0) cand_n[oi] = n_hit;
}

// One wave per outer tet: the pending (candidate, point) cases are queued in
// the wave's LDS slice across candidate chunks and tested in full rounds of
// 64; each result replaces its pending byte.
constexpr int kQueue = 320;  // < 64 left over + 4 * 64 appended per chunk

__global__ __launch_bounds__(256) void k_classify_exact(const double* tetX, const int32_t* outer_ids, int64_t n_outer,
                                                        double delta, const int64_t* cand_off, const int64_t* cand_n,
                                                        const int32_t* cand_m, uint32_t* cand_code) {
    __shared__ int64_t qp[4][kQueue];
    __shared__ uint8_t qk[4][kQueue];
    // the wave index is uniform: in a scalar register, the outer tet and its points are too
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    double P[4][3];
    load_outer_points(tetX, outer_ids[oi], P);
    const double d2 = delta * delta;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t* Q = qp[wave];
    uint8_t* K = qk[wave];
    auto run = [&](int j) {  // test queue item j (lane-private)
        const int64_t pos = Q[j];
        const int k = K[j];
        const double* Xg = tetX + 12 * (int64_t)cand_m[pos];
        double X[12];
        for (int e = 0; e < 12; ++e) X[e] = Xg[e];
        // byte k of the little-endian code word: a byte store, no atomic (the
        // other bytes may be written by other lanes at the same time)
        ((uint8_t*)cand_code)[4 * pos + k] = (uint8_t)classify_exact(X, P[k], d2);
    };
    const int64_t src = cand_off[oi], n = cand_n[oi];
    int nq = 0;
    for (int64_t j = 0; j < n; j += 64) {
        const int64_t pos = src + j + lane;
        const uint32_t code = (j + lane < n) ? cand_code[pos] : 0u;
        for (int k = 0; k < 4; ++k) {
            const bool pend = ((code >> (8 * k)) & 0xFFu) == kPending;
            const uint64_t bal = __ballot(pend);
            if (pend) {
                const int idx = nq + __popcll(bal & lt);
                Q[idx] = pos;
                K[idx] = (uint8_t)k;
            }
            nq += __popcll(bal);
        }
        wave_sync();
        while (nq >= 64) {
            run(lane);
            // move the rest of the queue down by 64
            int64_t keep_p[4];
            uint8_t keep_k[4];
            const int rest = nq - 64;
            for (int r = 0; r < 4; ++r) {
                const int from = 64 + lane + 64 * r;
                if (from < nq) {
                    keep_p[r] = Q[from];
                    keep_k[r] = K[from];
                }
            }
            wave_sync();
            for (int r = 0; r < 4; ++r) {
                const int to = lane + 64 * r;
                if (to < rest) {
                    Q[to] = keep_p[r];
                    K[to] = keep_k[r];
                }
            }
            wave_sync();
            nq = rest;
        }
    }
    if (lane < nq) run(lane);
}

// Class bytes of a candidate under a strategy, from the fullcaps classes
// (barycenter and inside are already final from the fast pass): nocaps
// drops CUT(0) (no T_I, no caps), overlap takes every element that meets
// the ball whole.
__device__ __forceinline__ uint32_t strategy_code(uint32_t code, int strategy) {
    if (strategy != S_NOCAPS && strategy != S_OVERLAP) return code;
    uint32_t out = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t cl = (code >> (8 * k)) & 0xFFu;
        if (strategy == S_NOCAPS) cl = cl == (uint32_t)C_CUT0 ? (uint32_t)C_OUT : cl;
        else cl = cl == (uint32_t)C_OUT ? (uint32_t)C_OUT : (uint32_t)C_IN;
        out |= cl << (8 * k);
    }
    return out;
}

// packed per-point class bytes -> 3-bit-per-point pair code
__device__ __forceinline__ uint32_t code12(uint32_t code) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c |= ((code >> (8 * k)) & 7u) << (3 * k);
    return c;
}

// which of the 4 outer points cut the tet (bit k set: class of point k is CUT)
__device__ __forceinline__ int cut_mask(uint32_t c12) {
    int mk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) mk |= ((((c12 >> (3 * k)) & 7u) >= (uint32_t)C_CUT0) ? 1 : 0) << k;
    return mk;
}

// the cut-mask buckets that some lane of the wave holds (bit b: mask b; mk < 0
// for no hit), the same in every lane
__device__ __forceinline__ uint32_t wave_buckets(int mk) {
    uint32_t bits = mk >= 0 ? 1u << mk : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bits |= (uint32_t)__shfl_xor((int)bits, off, 64);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)bits);
}

// Per outer tet: its hits per cut mask (which outer points cut the tet,
// cnt[16 oi + mask]) and per class over the four points (cls[5 oi + c - 1]
// for IN, CUT(0..3)).
__global__ __launch_bounds__(256) void k_pair_count(int64_t n_outer, const int64_t* cand_off, const int64_t* cand_n,
                                                    int strategy, const uint32_t* cand_code, int64_t* cnt,
                                                    uint32_t* cls) {
    // the wave index is uniform: in a scalar register, the outer tet and its points are too
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    const int64_t src = cand_off[oi], n = cand_n[oi];
    int64_t c[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    uint32_t q[5] = {0u, 0u, 0u, 0u, 0u};
    // four rounds of 64 candidates per step, their loads issued together
    for (int64_t j = 0; j < n; j += 4 * 64) {
        uint32_t ccs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ix = j + 64 * u + lane;
            ccs[u] = ix < n ? cand_code[src + ix] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ix = j + 64 * u + lane;
            const uint32_t cc = ix < n ? code12(strategy_code(ccs[u], strategy)) : 0u;
            const int mk = cc ? cut_mask(cc) : -1;
            const uint32_t held = wave_buckets(mk);
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (held & (1u << b)) c[b] += __popcll(__ballot(mk == b));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t cl = (cc >> (3 * k)) & 7u;
#pragma unroll
                for (int t = 0; t < 5; ++t) q[t] += cl == (uint32_t)(t + 1) ? 1u : 0u;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 5; ++t)
        for (int off = 32; off > 0; off >>= 1) q[t] += __shfl_xor(q[t], off, 64);
    int64_t v = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (b == lane) v = c[b];
    if (lane < 16) cnt[oi * 16 + lane] = v;
    if (lane < 5) {
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t)
            if (t == lane) w = q[t];
        cls[oi * 5 + lane] = w;
    }
}

// One wave per outer tet: the hits among its candidates, grouped by their cut
// mask (more cut points first, then the larger mask) and in candidate order
// within a group, to the final pair arrays.  Lanes of a wave then see the same
// cut points, so the sample loops of a wave are not run for points that only
// some lanes cut.
__global__ __launch_bounds__(256) void k_pair_compact(int64_t n_outer, const int64_t* cand_off, const int64_t* cand_n,
                                                      const int64_t* pair_off, const int64_t* cnt, int strategy,
                                                      const int32_t* cand_m, const uint32_t* cand_code, int32_t* pair_m,
                                                      uint16_t* pair_cls) {
    // the wave index is uniform: in a scalar register, the outer tet and its points are too
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t oi = (int64_t)blockIdx.x * 4 + wave;
    if (oi >= n_outer) return;
    const int64_t src = cand_off[oi], n = cand_n[oi];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    // group sizes (from k_pair_count) and starts, within the outer tet's list
    int c[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = (int)cnt[oi * 16 + b];
    // group order: 15 | 14 13 11 7 | 12 10 9 6 5 3 | 8 4 2 1 | 0
    const int order[16] = {15, 14, 13, 11, 7, 12, 10, 9, 6, 5, 3, 8, 4, 2, 1, 0};
    const int64_t p0 = pair_off[oi];
    int base[16];
    int run = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        base[order[i]] = run;
        run += c[order[i]];
    }
#pragma unroll
    for (int b = 0; b < 16; ++b) c[b] = 0;
    // four rounds of 64 candidates per step: their loads are issued together,
    // then the rounds are placed in candidate order
    for (int64_t j = 0; j < n; j += 4 * 64) {
        uint32_t ccs[4];
        int mks[4], ms[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ix = j + 64 * u + lane;
            ccs[u] = ix < n ? cand_code[src + ix] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ix = j + 64 * u + lane;
            ccs[u] = ix < n ? code12(strategy_code(ccs[u], strategy)) : 0u;
            mks[u] = ccs[u] ? cut_mask(ccs[u]) : -1;
            ms[u] = mks[u] >= 0 ? cand_m[src + ix] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t cc = ccs[u];
            const int mk = mks[u], m = ms[u];
            // only the buckets that some lane holds (a wave's candidates fall in a few)
            const uint32_t held = wave_buckets(mk);
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                if (!(held & (1u << b))) continue;
                const bool mine = mk == b;
                const uint64_t mask = __ballot(mine);
                if (mine) {
                    const int64_t pos = p0 + base[b] + c[b] + __popcll(mask & lt);
                    pair_m[pos] = m;
                    pair_cls[pos] = (uint16_t)cc;
                }
                c[b] += __popcll(mask);
            }
        }
    }
}

// pairs per outer tet (the sum of its 16 mask buckets), and the class totals
// of all pairs (one atomic per class and block into cls_tot[1..5])
__global__ __launch_bounds__(256) void k_pair_totals(const int64_t* cnt, const uint32_t* cls, int64_t n_outer,
                                                     int64_t* tot, unsigned long long* cls_tot) {
    __shared__ unsigned long long red[5][256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long q[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
    if (i < n_outer) {
        int64_t t = 0;
        for (int b = 0; b < 16; ++b) t += cnt[16 * i + b];
        tot[i] = t;
        for (int c = 0; c < 5; ++c) q[c] = cls[5 * i + c];
    }
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = q[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 5 && red[threadIdx.x][0]) atomicAdd(&cls_tot[1 + threadIdx.x], red[threadIdx.x][0]);
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
// its pair list.  When the vertex ids span at most 32 * kBitmapWords values
// (spatially ordered meshes: always), the set is a bitmap over that range,
// read out in ascending order through a block prefix sum of word popcounts;
// otherwise an LDS hash set sorted by a bitonic network.  The count pass
// writes |Ve| and, given a hand-off buffer (vbuf, vstride entries per outer
// tet), the set itself there, for k_ve_copy to move to ve_off; a set longer
// than vstride sets ERR_VEBUF and the fill pass builds the sets again at
// ve_off instead.
constexpr int kBitmapWords = 2048;

template <bool FILL>
__global__ __launch_bounds__(256) void k_pattern(const int32_t* tets, int64_t n_outer, const int64_t* pair_off,
                                                 const int32_t* pair_m, int hash_cap, int64_t* ucount,
                                                 const int64_t* ve_off, int32_t* ve_ids, int32_t* vbuf, int vstride,
                                                 unsigned* err) {
    extern __shared__ uint32_t hs[];
    __shared__ int sU, sLo, sHi;
    __shared__ int wsum[256];
    const uint32_t EMPTY = 0xFFFFFFFFu;
    const int64_t oi = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) {
        sU = 0;
        sLo = 0x7FFFFFFF;
        sHi = -1;
    }
    __syncthreads();
    const int64_t p0 = pair_off[oi], p1 = pair_off[oi + 1];
    int lo = 0x7FFFFFFF, hi = -1;
    for (int64_t p = p0 + t; p < p1; p += 256) {
        const int m = pair_m[p];
        for (int j = 0; j < 4; ++j) {
            const int v = tets[4 * (int64_t)m + j];
            lo = min(lo, v);
            hi = max(hi, v);
        }
    }
    atomicMin(&sLo, lo);
    atomicMax(&sHi, hi);
    __syncthreads();
    const int vlo = sLo;
    const int64_t range = (int64_t)sHi - (int64_t)vlo + 1;
    if (range > 0 && range <= 32 * (int64_t)kBitmapWords) {
        const int nw = (int)((range + 31) >> 5);
        for (int i = t; i < nw; i += 256) hs[i] = 0u;
        __syncthreads();
        for (int64_t p = p0 + t; p < p1; p += 256) {
            const int m = pair_m[p];
            for (int j = 0; j < 4; ++j) {
                const int r = tets[4 * (int64_t)m + j] - vlo;
                atomicOr(&hs[r >> 5], 1u << (r & 31));
            }
        }
        __syncthreads();
        // thread t owns words [t * cw, (t + 1) * cw)
        const int cw = (nw + 255) / 256;
        const int w0 = min(nw, t * cw), w1 = min(nw, (t + 1) * cw);
        int c = 0;
        for (int w = w0; w < w1; ++w) c += __popc(hs[w]);
        wsum[t] = c;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int add = t >= off ? wsum[t - off] : 0;
            __syncthreads();
            wsum[t] += add;
            __syncthreads();
        }
        const int U = wsum[255];
        int32_t* out;
        if (FILL) {
            out = ve_ids + ve_off[oi];
        } else {
            if (t == 0) ucount[oi] = U;
            if (!vbuf) return;
            if (U > vstride) {
                if (t == 0) atomicOr(err, ERR_VEBUF);
                return;
            }
            out = vbuf + oi * (int64_t)vstride;
        }
        int pos = wsum[t] - c;
        for (int w = w0; w < w1; ++w) {
            uint32_t bits = hs[w];
            while (bits) {
                const int bb = __ffs(bits) - 1;
                out[pos++] = vlo + 32 * w + bb;
                bits &= bits - 1u;
            }
        }
        return;
    }
    for (int i = t; i < hash_cap; i += 256) hs[i] = EMPTY;
    __syncthreads();
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
    int32_t* out;
    if (FILL) {
        out = ve_ids + ve_off[oi];
    } else {
        if (t == 0) ucount[oi] = U;
        if (!vbuf) return;
        if (U > vstride) {
            if (t == 0) atomicOr(err, ERR_VEBUF);
            return;
        }
        out = vbuf + oi * (int64_t)vstride;
    }
    for (int i = t; i < U; i += 256) out[i] = (int32_t)hs[i];
}

// the sets the count pass left in the hand-off buffer, to their place at ve_off
__global__ __launch_bounds__(256) void k_ve_copy(const int64_t* ve_off, const int32_t* vbuf, int vstride,
                                                 int32_t* ve_ids) {
    const int64_t oi = blockIdx.x;
    const int64_t b = ve_off[oi], U = ve_off[oi + 1] - b;
    const int32_t* src = vbuf + oi * (int64_t)vstride;
    for (int64_t i = threadIdx.x; i < U; i += 256) ve_ids[b + i] = src[i];
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

hipError_t launch_sorted_boxes(const double* tetX, const uint32_t* cell_tets, int64_t K, float4* box, double* sX,
                               hipStream_t s) {
    if (K <= 0) return hipSuccess;
    k_sorted_boxes<<<blocks_for(K), 256, 0, s>>>(tetX, cell_tets, K, box, sX);
    return hipGetLastError();
}

hipError_t launch_classify(const double* tetX, const int32_t* outer_ids, int64_t n_outer, const int64_t* cell_start,
                           const uint32_t* cell_tets, const float4* box, const double* sX, Grid g, double delta,
                           int strategy, const int64_t* cand_off, int64_t* cand_n, int64_t* cnt, uint32_t* cls,
                           int32_t* cand_m, uint32_t* cand_code, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_classify_fast<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(tetX, outer_ids, n_outer, cell_start, cell_tets, box,
                                                                  sX, g, delta, strategy, cand_off, cand_n, cand_m,
                                                                  cand_code);
    k_classify_exact<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(tetX, outer_ids, n_outer, delta, cand_off, cand_n,
                                                                    cand_m, cand_code);
    k_pair_count<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(n_outer, cand_off, cand_n, strategy, cand_code, cnt,
                                                               cls);
    return hipGetLastError();
}

hipError_t launch_pair_compact(int64_t n_outer, const int64_t* cand_off, const int64_t* cand_n, const int64_t* pair_off,
                               const int64_t* cnt, int strategy, const int32_t* cand_m, const uint32_t* cand_code,
                               int32_t* pair_m, uint16_t* pair_cls, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_pair_compact<<<(unsigned)((n_outer + 3) / 4), 256, 0, s>>>(n_outer, cand_off, cand_n, pair_off, cnt, strategy,
                                                                 cand_m, cand_code, pair_m, pair_cls);
    return hipGetLastError();
}

hipError_t launch_pair_totals(const int64_t* cnt, const uint32_t* cls, int64_t n_outer, int64_t* tot,
                              unsigned long long* cls_tot, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_pair_totals<<<blocks_for(n_outer), 256, 0, s>>>(cnt, cls, n_outer, tot, cls_tot);
    return hipGetLastError();
}

hipError_t launch_pattern(bool fill, const int32_t* tets, int64_t n_outer, const int64_t* pair_off,
                          const int32_t* pair_m, int hash_cap, int64_t* ucount, const int64_t* ve_off, int32_t* ve_ids,
                          int32_t* vbuf, int vstride, unsigned* err, hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    if (vbuf && vstride <= 0) return hipErrorInvalidValue;
    size_t sh = (size_t)(hash_cap > kBitmapWords ? hash_cap : kBitmapWords) * sizeof(uint32_t);
    if (fill)
        k_pattern<true><<<(unsigned)n_outer, 256, sh, s>>>(tets, n_outer, pair_off, pair_m, hash_cap, ucount, ve_off,
                                                          ve_ids, nullptr, 0, err);
    else
        k_pattern<false><<<(unsigned)n_outer, 256, sh, s>>>(tets, n_outer, pair_off, pair_m, hash_cap, ucount,
                                                           ve_off, ve_ids, vbuf, vstride, err);
    return hipGetLastError();
}

hipError_t launch_ve_copy(int64_t n_outer, const int64_t* ve_off, const int32_t* vbuf, int vstride, int32_t* ve_ids,
                          hipStream_t s) {
    if (n_outer <= 0) return hipSuccess;
    k_ve_copy<<<(unsigned)n_outer, 256, 0, s>>>(ve_off, vbuf, vstride, ve_ids);
    return hipGetLastError();
}

}  // namespace nlfem
