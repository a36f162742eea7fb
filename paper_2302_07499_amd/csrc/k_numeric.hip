// Numeric phase: per-pair inner integrals (fullcaps) and their reduction per
// outer tet.
//
// Decomposition of the pair contribution (main assembly algorithm, Sec. 4.3):
// with a_u(y) = phi_(m,u)(y) - phi_(n,u)(p) and the moments S0, S1, S2 of the
// inner tet's barycentric coordinates over E_m n B_{delta,h}(p),
//   K_uv = f_m psi w [S2_uv - c_u S1_v - c_v S1_u + c_u c_v S0]
// (c = the outer rule row of p, f_m = 1 on T_Omega, 2 on T_OmegaI).  Summed
// over the pairs, the c c^T S0 terms only need T0_k = sum_m f_m S0 per outer
// point, the cross terms only R_k(v) = sum_{m containing v} f_m S1_v per
// (outer point, vertex), and the S2 terms only the per-inner-tet sum
// G_m = sum_q psi f_m w_q S2 (needed on T_Omega only: T_OmegaI rows carry no
// unknowns).  T0 and R are reduced inside the outer tet's workgroup and
// leave it as the cross block C^n[i][j] = -psi w sum_k c_kj R_k(Ve_i) and the
// outer block O^n[j][j'] = psi w sum_k c_kj c_kj' T0_k.  G_m is summed in
// global two-word fixed-point accumulators: the Monte Carlo / subdivision
// part of cut points directly, inside points as a count weight times the
// closed-form 4-point-rule moments of E_m (k_rows.hip).
#include "device_geom.hpp"

#ifndef NLFEM_INTEGRATE_WAVES
#define NLFEM_INTEGRATE_WAVES 3  // minimum waves per SIMD requested for k_integrate (register cap)
#endif

namespace nlfem {

namespace {

// x is added to a two-word fixed-point sum: the coarse word counts units of
// 2^-s, the fine word the remainder in units of 2^-(s+48), both two's
// complement.  The pair (h, l) of one term is the integer nearest to
// x 2^(s+48) split at bit 48: h the integer nearest to x 2^s, l the integer
// nearest to the remainder times 2^48 (|l| <= 2^47).  Integer sums are
// order-independent, so the result is deterministic, and the fine word keeps
// small contributions (thin cut slivers) relatively exact.
constexpr int FX_LO_BITS = 48;
// Adding 1.5 2^52 to |v| < 2^51 rounds v to an integer (to nearest, ties to
// even) held in the low mantissa bits, which the bit difference reads out.
constexpr double kRoundMagic = 6755399441055744.0;

// needs |x 2^s| < 2^51 (the plan's scales keep every single term below it)
__device__ __forceinline__ void fx_split(double x, double fx, unsigned long long& hi, unsigned long long& lo) {
    const double xs = x * fx;                    // exact: fx is a power of two
    const double t = xs + kRoundMagic;           // kRoundMagic + nearest integer to xs
    const double r = xs - (t - kRoundMagic);     // exact, |r| <= 1/2
    const double u = fma(r, 281474976710656.0, kRoundMagic);  // nearest integer to r 2^48, |.| <= 2^47
    hi = (unsigned long long)(__double_as_longlong(t) - __double_as_longlong(kRoundMagic));
    lo = (unsigned long long)(__double_as_longlong(u) - __double_as_longlong(kRoundMagic));
}

__device__ __forceinline__ void fx_add(unsigned long long* hi, unsigned long long* lo, double x, double fx) {
    unsigned long long h, l;
    fx_split(x, fx, h, l);
    atomicAdd(hi, h);
    atomicAdd(lo, l);
}

// carry-normalised: the fine word is reduced to [0, 2^48) first (its carry,
// an arithmetic shift, goes to the coarse word), so both conversions are
// exact for totals below 2^53 coarse units
__device__ __forceinline__ double fx_value(unsigned long long hi, unsigned long long lo, int shift) {
    const unsigned long long h = hi + (unsigned long long)((long long)lo >> FX_LO_BITS);
    const double v = (double)(lo & ((1ull << FX_LO_BITS) - 1ull)) * 0x1p-48 + (double)(long long)h;
    return ldexp(v, -shift);
}

// the same two-word sums in global memory (the G_m accumulators)
__device__ __forceinline__ void fxs_add_global(unsigned long long* hi, unsigned long long* lo, double x, double fx) {
    fx_add(hi, lo, x, fx);
}

// Cut (pair, outer point) items are taken in chunks of kChunk pairs.
constexpr int kChunk = 256;
// LDS beyond R, T0 and the per-thread T0 words: the chunk's item prefix sums
// (kChunk + 1 ints, padded to 8 bytes) and its pairs' local vertex positions
// (kChunk x 4 u16), before Ve
constexpr size_t kChunkLds =
    ((size_t)(kChunk + 1) * 4 + 7) / 8 * 8 + (size_t)kChunk * 8 + (size_t)kChunk * 4 * 2 + (size_t)kChunk * 6;

// One workgroup of BLOCK threads integrates one outer tet.  LDS: R [4][umax]
// and T0 [4] as two-word fixed-point sums (coarse words, then fine words),
// each thread's own T0 words [4][2][BLOCK] (every fold of a wave targets the
// same T0[k], so the threads sum privately and the block adds the slots up at
// the end: the same integers, without same-address atomics), the chunk
// tables, Ve [umax], and the 4 outer points.  A is IntegrateArgs, or the same
// type in the constant address space for descriptors read from a device
// table.  OPAQUE_TID hides the thread index behind an empty asm so that a
// caller's loop cannot hoist the per-thread addresses out of it (they would
// stay live across the whole item loop of a persistent kernel and spill).
//
// The pair list is walked in chunks of kChunk pairs.  First each thread takes
// whole pairs: their inside points are folded at once and their cut points
// counted.  Then the chunk's cut points are enumerated as (pair, point) items
// through a prefix sum, and lane it of the workgroup takes item it: one cut
// setup and one sample loop per lane, so a wave's lanes are all busy whatever
// the mix of cut masks (one thread per pair looping over its cut points keeps
// a fifth of them idle).  Items of one pair sit in neighbouring lanes; their
// S2 sums for G_m are added across those lanes (a fixed tree over at most
// four lanes, by item index modulo 64 and chunk, so independent of BLOCK)
// and sent to the global accumulators once per pair and wave.
// GR: the R sums in global memory (a.rglob) and Ve read from global memory,
// for local vertex sets too large for LDS; the same integers either way.
template <typename T, int BLOCK, bool VR, int KEY, typename A, bool OPAQUE_TID = false, bool GR = false>
__device__ __forceinline__ void integrate_outer(const A& a, int64_t oi, unsigned long long* smem64,
                                                double (*P)[3]) {
    const int umax = GR ? 0 : a.umax;           // LDS words per R row
    unsigned long long* R = smem64;             // coarse [4][umax] (LDS mode)
    unsigned long long* Rl = R + 4 * umax;      // fine   [4][umax] (LDS mode)
    unsigned long long* T0 = Rl + 4 * umax;     // coarse [4]
    unsigned long long* T0l = T0 + 4;           // fine   [4]
    unsigned long long* T0p = T0l + 4;          // per thread [4][2][BLOCK]
    int32_t* cs = (int32_t*)(T0p + 8 * BLOCK);  // [kChunk + 1] item prefix sums of the chunk
    uint16_t* lvs = (uint16_t*)((char*)cs + (kChunkLds - (size_t)kChunk * 22));  // [kChunk][4]
    uint16_t* ipair = lvs + 4 * kChunk;  // [4 kChunk] per item: its pair's chunk position (| point << 14)
    int32_t* pm = (int32_t*)(ipair + 4 * kChunk);  // [kChunk] inner tet of each pair
    uint16_t* pcl = (uint16_t*)(pm + kChunk);      // [kChunk] class code | T_Omega << 15
    int32_t* ve_lds = (int32_t*)((char*)cs + kChunkLds);
    const int n = a.outer_ids[oi];
    const int64_t vb = a.ve_off[oi];
    const int U = (int)(a.ve_off[oi + 1] - vb);
    unsigned long long* rg = GR ? a.rglob + 8 * vb : nullptr;  // [U][8] (global mode)
    const int32_t* ve = GR ? a.ve_ids + vb : ve_lds;
    // coarse and fine word of R_k at local vertex position i
    auto rco = [&](int k, int i) { return GR ? rg + 8 * i + k : R + k * umax + i; };
    auto rfi = [&](int k, int i) { return GR ? rg + 8 * i + 4 + k : Rl + k * umax + i; };
    int t = threadIdx.x;
    if constexpr (OPAQUE_TID) asm volatile("" : "+v"(t));
    if constexpr (GR) {
        for (int i = t; i < 8 * U; i += BLOCK) rg[i] = 0ull;
    } else {
        for (int i = t; i < U; i += BLOCK) ve_lds[i] = a.ve_ids[vb + i];
        for (int i = t; i < 8 * umax; i += BLOCK) R[i] = 0ull;
    }
    for (int i = 0; i < 8; ++i) T0p[i * BLOCK + t] = 0ull;
    if (t < 4) {
        double Xn[12];
        for (int i = 0; i < 12; ++i) Xn[i] = a.tetX[12 * (int64_t)n + i];
        outer_point(Xn, t, P[t]);
    }
    const double w = a.vol[n] * 0.25;
    const double pw = a.psi * w;
    const int64_t ks = a.gstride;
    __syncthreads();
    const double d2 = a.delta * a.delta;
    const double fx = ldexp(1.0, a.fx_shift);
    const double gfx = ldexp(1.0, a.g_shift);
    const double wfx = ldexp(1.0, a.w_shift);
    const int lane = t & 63;
    // folds S0, S1 of outer point k's moments into T0 and R (lv: local
    // positions of the inner tet's vertices in Ve, all present)
    auto fold = [&](int k, const double* S, const int* lv, double fm) {
        {
            unsigned long long h, l;
            fx_split(fm * S[0], fx, h, l);
            T0p[(2 * k) * BLOCK + t] += h;
            T0p[(2 * k + 1) * BLOCK + t] += l;
        }
        for (int j = 0; j < 4; ++j)
            if (lv[j] < U) fx_add(rco(k, lv[j]), rfi(k, lv[j]), fm * S[1 + j], fx);
    };
    const int64_t p0 = a.pair_off[oi], p1 = a.pair_off[oi + 1];
    int ustep = 1;  // the largest power of two <= U (1 when U = 0)
    while (2 * ustep <= U) ustep *= 2;
    for (int64_t c0 = p0; c0 < p1; c0 += kChunk) {
        const int nc = (int)(p1 - c0 < (int64_t)kChunk ? p1 - c0 : (int64_t)kChunk);
        // (a) whole pairs: inside points, cut-point counts, local vertex positions
        for (int i = t; i < kChunk; i += BLOCK) {
            int ncut = 0;
            if (i < nc) {
                const int64_t p = c0 + i;
                const int m = a.pair_m[p];
                const uint32_t code = a.pair_cls[p];
                // the four positions by one lock-step binary search (Ve is sorted):
                // lv[j] = the number of entries below vertex j, each step's four
                // reads independent of each other
                int lv[4] = {0, 0, 0, 0};
                int32_t key[4];
                for (int j = 0; j < 4; ++j) key[j] = a.tets[4 * (int64_t)m + j];
                for (int step = ustep; step > 0; step >>= 1) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (lv[j] + step <= U && ve[lv[j] + step - 1] < key[j]) lv[j] += step;
                }
                for (int j = 0; j < 4; ++j) lvs[4 * i + j] = (uint16_t)lv[j];
                const bool omega = a.region[m] != 0;
                if constexpr (KEY == 0) {
                    pm[i] = m;
                    pcl[i] = (uint16_t)(code | (omega ? 0x8000u : 0u));
                }
                int n_in = 0;
#pragma unroll 1
                for (int k = 0; k < 4; ++k) {
                    const int c = (int)((code >> (3 * k)) & 7u);
                    if (c == C_IN) {
                        double S[15];
                        in_moments(a.vol[m], S);
                        fold(k, S, lv, omega ? 1.0 : 2.0);
                        ++n_in;
                    }
                    ncut += c >= C_CUT0 ? 1 : 0;
                }
                if (omega && n_in) {
                    unsigned long long* ga = a.gacc + (int64_t)m;
                    fxs_add_global(&ga[20 * ks], &ga[21 * ks], pw * (double)n_in, wfx);
                }
            }
            cs[i] = ncut;
        }
        __syncthreads();
        // exclusive prefix sum of the counts (one wave; four entries per lane)
        if (t < 64) {
            const int v0 = cs[4 * t], v1 = cs[4 * t + 1], v2 = cs[4 * t + 2], v3 = cs[4 * t + 3];
            const int sum = ((v0 + v1) + v2) + v3;
            int incl = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const int o = __shfl_up(incl, off, 64);
                if (t >= off) incl += o;
            }
            const int ex = incl - sum;
            cs[4 * t] = ex;
            cs[4 * t + 1] = ex + v0;
            cs[4 * t + 2] = ex + v0 + v1;
            cs[4 * t + 3] = ex + v0 + v1 + v2;
            if (t == 63) cs[kChunk] = incl;
        }
        __syncthreads();
        // each pair lists its items (pair position, cut point), so that an item
        // finds both in one read
        for (int i = t; i < nc; i += BLOCK) {
            if constexpr (KEY == 0) {
                const uint32_t code = pcl[i];
                int q = cs[i];
                for (int kk = 0; kk < 4; ++kk)
                    if (((code >> (3 * kk)) & 7u) >= (uint32_t)C_CUT0) ipair[q++] = (uint16_t)(i | (kk << 14));
            } else {
                for (int q = cs[i]; q < cs[i + 1]; ++q) ipair[q] = (uint16_t)i;
            }
        }
        __syncthreads();
        const int n_items = cs[kChunk];
        // (b) the chunk's cut (pair, point) items, one per lane
        for (int ib = 0; ib < n_items; ib += BLOCK) {
            const int it = ib + t;
            const bool valid = it < n_items;
            int pi = -1;
            double g[10];
            for (int i = 0; i < 10; ++i) g[i] = 0.0;
            int m = 0;
            bool omega = false;
            if (valid) {
                // pair keying takes the pair's tet, class and the item's cut point
                // from LDS; element keying reads them again (its table-fed sample
                // loop measured faster with the register allocation this gives)
                int k;
                if constexpr (KEY == 0) {
                    const uint32_t ik = ipair[it];
                    pi = (int)(ik & 0x3FFFu);
                    k = (int)(ik >> 14);
                    m = pm[pi];
                    omega = (pcl[pi] & 0x8000u) != 0;
                } else {
                    pi = ipair[it];
                    const int64_t p = c0 + pi;
                    m = a.pair_m[p];
                    const uint32_t code = a.pair_cls[p];
                    unsigned cm = 0u;
                    for (int kk = 0; kk < 4; ++kk)
                        cm |= (((code >> (3 * kk)) & 7u) >= (uint32_t)C_CUT0 ? 1u : 0u) << kk;
                    k = nth_bit(cm, it - cs[pi]);
                    omega = a.region[m] != 0;
                }
                const double volm = a.vol[m];
                int lv[4];
                for (int j = 0; j < 4; ++j) lv[j] = lvs[4 * pi + j];
                const double* X = a.tetX + 12 * (int64_t)m;
                CutGeom cg;
                double D[5];
                CornerGeom cr;
                double S[15];
                cut_det<T>(X, volm, P[k], d2, cg, D, g, VR ? &cr : nullptr);
                if (a.caps) {
                    cut_mc<T, VR, KEY>(X, volm, P[k], d2, cg, a.mc_samples, a.key0, a.key1, (uint32_t)(4 * n + k),
                                       (uint32_t)m, S, &cr, a.stab ? a.stab + (int64_t)m * a.stab_stride : nullptr);
                } else {
                    for (int i = 0; i < 15; ++i) S[i] = 0.0;  // nocaps: the subdivision T_I only
                }
                for (int i = 0; i < 5; ++i) S[i] = D[i] + S[i];
                fold(k, S, lv, omega ? 1.0 : 2.0);
                for (int i = 0; i < 10; ++i) g[i] += S[5 + i];
            }
            // G_m: the items of one pair (at most four neighbouring lanes) summed
            // over the lanes, then sent by the pair's first lane in the wave
            const bool gl = valid && omega;
#pragma unroll
            for (int off = 1; off <= 2; off <<= 1) {
                const int opi = __shfl_down(pi, off, 64);
                const int og = __shfl_down(gl ? 1 : 0, off, 64);
                const bool take = gl && lane + off < 64 && og && opi == pi;
#pragma unroll
                for (int i = 0; i < 10; ++i) {
                    const double o = __shfl_down(g[i], off, 64);
                    if (take) g[i] += o;
                }
            }
            const int ppi = __shfl_up(pi, 1, 64);
            if (gl && (lane == 0 || ppi != pi)) {
                unsigned long long* ga = a.gacc + (int64_t)m;
                for (int i = 0; i < 10; ++i) fxs_add_global(&ga[(2 * i) * ks], &ga[(2 * i + 1) * ks], pw * g[i], gfx);
            }
        }
        __syncthreads();
    }
    if (t < 8) {
        unsigned long long v = 0ull;
        for (int i = 0; i < BLOCK; ++i) v += T0p[t * BLOCK + i];
        if (t & 1) T0l[t >> 1] = v;
        else T0[t >> 1] = v;
    }
    __syncthreads();
    const int sh = a.fx_shift;
    // cross block [Ve_i][j] = -psi w sum_k c_kj R_k(Ve_i)
    double* cb = a.cblk + 4 * vb;
    for (int r = t; r < 4 * U; r += BLOCK) {
        const int i = r >> 2, j = r & 3;
        double cR = 0.0;
        for (int k = 0; k < 4; ++k) cR += rule_w(k, j) * fx_value(*rco(k, i), *rfi(k, i), sh);
        cb[r] = -(pw * cR);
    }
    // outer block and load vector (sum_k w c_kj f(p_k))
    double* ob = a.oblk + 20 * oi;
    if (t < 16) {
        const int j = t >> 2, jj = t & 3;
        double O = 0.0;
        for (int k = 0; k < 4; ++k) O += (rule_w(k, j) * rule_w(k, jj)) * fx_value(T0[k], T0l[k], sh);
        ob[t] = pw * O;
    } else if (t < 20) {
        const int j = t - 16;
        double f = 0.0;
        if (a.f_qp)
            for (int k = 0; k < 4; ++k) f += (w * rule_w(k, j)) * a.f_qp[4 * (int64_t)n + k];
        ob[t] = f;
    }
}

template <typename T, int BLOCK, bool VR, int KEY, typename A, bool OPAQUE_TID = false>
__device__ __forceinline__ void integrate_any(const A& a, int64_t oi, unsigned long long* smem64, double (*P)[3]) {
    integrate_outer<T, BLOCK, VR, KEY, A, OPAQUE_TID>(a, oi, smem64, P);
}

// Local vertex sets beyond LDS: the R sums in global memory, one (pair, cut
// point) item per lane for either keying.
template <typename T, bool VR, int KEY>
__global__ __launch_bounds__(256, NLFEM_INTEGRATE_WAVES) void k_integrate_global(IntegrateArgs a) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    integrate_outer<T, 256, VR, KEY, IntegrateArgs, false, true>(a, (int64_t)blockIdx.x, smem64, P);
}

// VR: the caps of cut pairs with n_in >= 1 are sampled on E_m minus U_I;
// KEY: pair (0) or element (1) keying of the Monte Carlo samples
#ifndef NLFEM_XCD_CHUNK
#define NLFEM_XCD_CHUNK 64
#endif
// Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b mod 8).
// Runs of C consecutive outer tets (neighbours in the mesh order, so their
// balls share inner tets) go to one XCD and its L2: workgroup b takes outer
// position ((b / 8) / C) 8 C + (b mod 8) C + (b / 8) mod C; the tail past the
// last whole group of 8 C keeps its own position.
__device__ __forceinline__ int64_t xcd_outer_pos(int64_t b, int64_t G) {
    constexpr int64_t C = NLFEM_XCD_CHUNK;
    if constexpr (C <= 1) return b;
    const int64_t full = G / (8 * C) * (8 * C);
    if (b >= full) return b;
    const int64_t x = b & 7, local = b >> 3;
    return (local / C) * (8 * C) + x * C + local % C;
}

template <typename T, bool VR, int KEY>
__global__ __launch_bounds__(256, NLFEM_INTEGRATE_WAVES) void k_integrate(IntegrateArgs a) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    integrate_any<T, 256, VR, KEY>(a, xcd_outer_pos((int64_t)blockIdx.x, (int64_t)gridDim.x), smem64, P);
}

// descriptors of a batch are read-only for the whole launch: read through the
// constant address space so that they load into scalar registers, and can be
// loaded again instead of being held, as kernel arguments are
typedef const __attribute__((address_space(4))) IntegrateArgs ConstArgs;

// Persistent batched integration: a grid sized to the machine pulls work
// items (mesh, outer position) from a device queue, longest first, until it
// is empty; each item's results depend on the item only.
template <typename T, int BLOCK, bool VR, int KEY>
__global__ __launch_bounds__(BLOCK, NLFEM_INTEGRATE_WAVES) void k_integrate_batch(const IntegrateArgs* descs,
                                                                                 const int2* items, int64_t n_items,
                                                                                 unsigned long long* head) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    __shared__ long long cur;
    while (true) {
        if (threadIdx.x == 0) cur = (long long)atomicAdd(head, 1ull);
        __syncthreads();
        const long long it = cur;
        __syncthreads();
        if (it >= n_items) break;
        // the item and its descriptor are the same for the whole workgroup
        const int2 item = items[__builtin_amdgcn_readfirstlane((int)it)];
        const int mesh = __builtin_amdgcn_readfirstlane(item.x);
        const int pos = __builtin_amdgcn_readfirstlane(item.y);
        ConstArgs* d = (ConstArgs*)(descs + mesh);
        integrate_any<T, BLOCK, VR, KEY, ConstArgs, true>(*d, (int64_t)pos, smem64, P);
        __syncthreads();
    }
}

__global__ void k_reset_u64(unsigned long long* p) { *p = 0ull; }

// One workgroup per work item (mesh, outer position), in list order: the
// dispatcher starts workgroups in increasing index as slots free up, so a
// longest-first list is taken longest first without a software queue.
template <typename T, int BLOCK, bool VR, int KEY>
__global__ __launch_bounds__(BLOCK, NLFEM_INTEGRATE_WAVES) void k_integrate_items(const IntegrateArgs* descs,
                                                                                 const int2* items) {
    extern __shared__ unsigned long long smem64[];
    __shared__ double P[4][3];
    const int2 item = items[blockIdx.x];
    const int mesh = __builtin_amdgcn_readfirstlane(item.x);
    const int pos = __builtin_amdgcn_readfirstlane(item.y);
    ConstArgs* d = (ConstArgs*)(descs + mesh);
    integrate_any<T, BLOCK, VR, KEY>(*d, (int64_t)pos, smem64, P);
}


// Paper-exact right-hand side (eq. Fh with g at the inner points, eq. F1.5):
// the load terms of each outer tet gain
//   sum_k w c_kj 2 psi sum_{E_m in T_Omega_I} int_{E_m n B_delta,h(p_k)} (g - g_h),
// g_h the nodal interpolant that the constraint columns already carry.  One
// workgroup per outer tet, after the integration (which writes the load
// terms) and before the row assembly; the per-point sums are reduced in a
// fixed order, so the result is reproducible.
constexpr int kExactGBlock = 256;
template <int DEG>
__global__ __launch_bounds__(kExactGBlock, 2) void k_exact_g(IntegrateArgs a, const double* g_nodal, const double* coef) {
    // coefficients through the constant address space: scalar loads that the
    // compiler may repeat instead of holding them in vector registers
    typedef const __attribute__((address_space(4))) double ConstCoef;
    ConstCoef* cf = (ConstCoef*)coef;
    __shared__ double P[4][3];
    __shared__ double red[4][kExactGBlock];
    const int64_t oi = blockIdx.x;
    const int n = a.outer_ids[oi];
    const int t = threadIdx.x;
    if (t < 4) {
        double Xn[12];
        for (int i = 0; i < 12; ++i) Xn[i] = a.tetX[12 * (int64_t)n + i];
        outer_point(Xn, t, P[t]);
    }
    __syncthreads();
    const double d2 = a.delta * a.delta;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = a.pair_off[oi] + t; p < a.pair_off[oi + 1]; p += kExactGBlock) {
        const int m = a.pair_m[p];
        if (a.region[m]) continue;  // T_Omega inner elements carry no g
        const uint32_t code = a.pair_cls[p];
        const double* X = a.tetX + 12 * (int64_t)m;
        double gv[4];
        for (int l = 0; l < 4; ++l) gv[l] = g_nodal ? g_nodal[a.tets[4 * (int64_t)m + l]] : 0.0;
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int c = (int)((code >> (3 * k)) & 7u);
            if (c == C_OUT) continue;
            acc[k] += pair_g_defect<DEG>(X, a.vol[m], P[k], d2, c, a.mc_samples, a.caps != 0, a.keying, a.key0, a.key1,
                                         (uint32_t)(4 * n + k), (uint32_t)m, gv, cf);
        }
    }
    for (int k = 0; k < 4; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int h = kExactGBlock / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + h];
        __syncthreads();
    }
    if (t < 4) {
        const double w = a.vol[n] * 0.25;
        double add = 0.0;
        for (int k = 0; k < 4; ++k) add += (w * rule_w(k, t)) * ((2.0 * a.psi) * red[k][0]);
        a.oblk[20 * oi + 16 + t] += add;
    }
}

// per-pair moments for outer positions [o_lo, o_hi): slot (p - pair_off[o_lo])*4 + k
template <typename T, bool VR, int KEY>
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
        const double* X = a.tetX + 12 * (int64_t)m;
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            const int c = (int)((code >> (3 * k)) & 7u);
            const int64_t idx = (p - base) * 4 + k;
            out_qm[3 * idx] = 4 * n + k;
            out_qm[3 * idx + 1] = m;
            out_qm[3 * idx + 2] = c;
            if (c == C_OUT) continue;
            double S[15];
            pair_moments<T, VR, KEY>(X, a.vol[m], P[k], d2, c, a.mc_samples, a.caps != 0, a.key0, a.key1,
                                     (uint32_t)(4 * n + k), (uint32_t)m, S);
            for (int i = 0; i < 15; ++i) out_S[15 * idx + i] = S[i];
        }
    }
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

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t integrate_lds_bytes(int umax) {
    return (size_t)umax * 68 + 64 + 8 * 256 * sizeof(unsigned long long) + kChunkLds;
}
size_t integrate_global_lds_bytes() { return 64 + 8 * 256 * sizeof(unsigned long long) + kChunkLds; }

// kernel selection over (precision, cap sampling, keying)
#define NLFEM_DISPATCH3(fp32, vr, key, LAUNCH)                 \
    do {                                                        \
        if (vr) {                                               \
            if (key) {                                          \
                if (fp32) LAUNCH(float, true, 1);               \
                else LAUNCH(double, true, 1);                   \
            } else {                                            \
                if (fp32) LAUNCH(float, true, 0);               \
                else LAUNCH(double, true, 0);                   \
            }                                                   \
        } else {                                                \
            if (key) {                                          \
                if (fp32) LAUNCH(float, false, 1);              \
                else LAUNCH(double, false, 1);                  \
            } else {                                            \
                if (fp32) LAUNCH(float, false, 0);              \
                else LAUNCH(double, false, 0);                  \
            }                                                   \
        }                                                       \
    } while (0)

// The element-keyed samples of every element (mc_philox<1>, two per call),
// packed; the padding words past N are zero and never used.
__global__ __launch_bounds__(256) void k_sample_table(int64_t K, int N, int64_t stride, uint32_t key0, uint32_t key1,
                                                      unsigned long long* tab) {
    const int64_t half = stride >> 1;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= K * half) return;
    const int64_t m = t / half;
    const int j = (int)(t - m * half);
    unsigned long long out[2] = {0ull, 0ull};
    if (2 * j < N) {
        uint32_t w[4];
        mc_philox<1>(0u, (uint32_t)m, (uint32_t)j, key0, key1, w);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (2 * j + h < N) {
                uint32_t L[4];
                lambda_u(w, h, L);
                out[h] = pack_lambda(L);
            }
        }
    }
    ulonglong2 v;
    v.x = out[0];
    v.y = out[1];
    *(ulonglong2*)(tab + m * stride + 2 * j) = v;
}

hipError_t launch_sample_table(int64_t K, int N, int64_t stride, uint32_t key0, uint32_t key1,
                               unsigned long long* tab, hipStream_t s) {
    if (K <= 0 || N <= 0) return hipSuccess;
    // rows of `stride` words: the N samples, the padding the sample loop reads ahead
    if (stride < sample_table_stride(N) || (stride & 1)) return hipErrorInvalidValue;
    const int64_t n = K * (stride >> 1);
    k_sample_table<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(K, N, stride, key0, key1, tab);
    return hipGetLastError();
}

hipError_t launch_integrate(const IntegrateArgs& a, bool fp32, hipStream_t s) {
    if (a.n_outer <= 0) return hipSuccess;
    const unsigned g = (unsigned)a.n_outer;
    if (a.rglob) {
        const size_t sh = integrate_global_lds_bytes();
#define L_GLB(T, VR, KEY) k_integrate_global<T, VR, KEY><<<g, 256, sh, s>>>(a)
        NLFEM_DISPATCH3(fp32, a.vr, a.keying, L_GLB);
#undef L_GLB
        return hipGetLastError();
    }
    size_t sh = integrate_lds_bytes(a.umax);
#define L_ONE(T, VR, KEY) k_integrate<T, VR, KEY><<<g, 256, sh, s>>>(a)
    NLFEM_DISPATCH3(fp32, a.vr, a.keying, L_ONE);
#undef L_ONE
    return hipGetLastError();
}

hipError_t launch_integrate_batch(const IntegrateArgs* descs, const int2* items, int64_t n_items,
                                  unsigned long long* head, int umax, bool fp32, bool vr, int keying, int block,
                                  int grid, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (n_items > 0x7fffffff || grid <= 0) return hipErrorInvalidValue;
    const size_t sh = integrate_lds_bytes(umax);
    // a fill kernel, not a memset: the launch is captured in a graph
    k_reset_u64<<<1, 1, 0, s>>>(head);
    const unsigned g = (unsigned)grid;
    if (block == 128) {
#define L_B128(T, VR, KEY) k_integrate_batch<T, 128, VR, KEY><<<g, 128, sh, s>>>(descs, items, n_items, head)
        NLFEM_DISPATCH3(fp32, vr, keying, L_B128);
#undef L_B128
    } else {
#define L_B256(T, VR, KEY) k_integrate_batch<T, 256, VR, KEY><<<g, 256, sh, s>>>(descs, items, n_items, head)
        NLFEM_DISPATCH3(fp32, vr, keying, L_B256);
#undef L_B256
    }
    return hipGetLastError();
}

hipError_t launch_integrate_items(const IntegrateArgs* descs, const int2* items, int64_t n_items, int umax, bool fp32,
                                  bool vr, int keying, int block, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (n_items > 0x7fffffff) return hipErrorInvalidValue;
    const size_t sh = integrate_lds_bytes(umax);
    const unsigned g = (unsigned)n_items;
    if (block == 128) {
#define L_I128(T, VR, KEY) k_integrate_items<T, 128, VR, KEY><<<g, 128, sh, s>>>(descs, items)
        NLFEM_DISPATCH3(fp32, vr, keying, L_I128);
#undef L_I128
    } else {
#define L_I256(T, VR, KEY) k_integrate_items<T, 256, VR, KEY><<<g, 256, sh, s>>>(descs, items)
        NLFEM_DISPATCH3(fp32, vr, keying, L_I256);
#undef L_I256
    }
    return hipGetLastError();
}

hipError_t launch_debug_pairs(const IntegrateArgs& a, bool fp32, int64_t o_lo, int64_t o_hi, double* out_S,
                              int32_t* out_qm, hipStream_t s) {
    if (o_hi <= o_lo) return hipSuccess;
    const unsigned g = (unsigned)(o_hi - o_lo);
#define L_DBG(T, VR, KEY) k_debug_pairs<T, VR, KEY><<<g, 256, 0, s>>>(a, o_lo, out_S, out_qm)
    NLFEM_DISPATCH3(fp32, a.vr, a.keying, L_DBG);
#undef L_DBG
    return hipGetLastError();
}

hipError_t launch_exact_g(const IntegrateArgs& a, const double* g_nodal, const double* coef, int deg, hipStream_t s) {
    if (a.n_outer <= 0) return hipSuccess;
    if (deg < 0 || deg > kMaxGDegree || a.vr) return hipErrorInvalidValue;
    const unsigned g = (unsigned)a.n_outer;
    switch (deg) {
        case 0: k_exact_g<0><<<g, kExactGBlock, 0, s>>>(a, g_nodal, coef); break;
        case 1: k_exact_g<1><<<g, kExactGBlock, 0, s>>>(a, g_nodal, coef); break;
        case 2: k_exact_g<2><<<g, kExactGBlock, 0, s>>>(a, g_nodal, coef); break;
        case 3: k_exact_g<3><<<g, kExactGBlock, 0, s>>>(a, g_nodal, coef); break;
        default: k_exact_g<4><<<g, kExactGBlock, 0, s>>>(a, g_nodal, coef); break;
    }
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


}  // namespace nlfem
