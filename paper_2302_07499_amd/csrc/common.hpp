// Internal declarations shared by the host runtime and the kernel files of
// the nlfem library.  Not part of the public C ABI (include/nlfem.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace nlfem {

// pair class codes (3 bits per outer point in the packed per-pair word)
enum : int { C_OUT = 0, C_IN = 1, C_CUT0 = 2 };
// ball approximation strategies (nlfem_strategy)
enum : int { S_FULLCAPS = 0, S_NOCAPS = 1, S_OVERLAP = 2, S_INSIDE = 3, S_BARYCENTER = 4 };

// 4-point degree-2 rule: node r has barycentric alpha on vertex r, beta on
// the others; alpha = (5 + 3 sqrt 5) / 20, beta = (5 - sqrt 5) / 20 rounded
// to double.
constexpr double kAlpha = 0x1.2bbae2a27f932p-1;
constexpr double kBeta = 0x1.1b06d1d200913p-3;

// exact-g right-hand side: tensor polynomial degree per axis, coefficients
constexpr int kMaxGDegree = 4;
constexpr int kMaxGCoef = (kMaxGDegree + 1) * (kMaxGDegree + 1) * (kMaxGDegree + 1);

// Uniform grid over tet bounding-box minimum corners (see k_plan.hip).
struct Grid {
    double ox, oy, oz;  // origin
    double cs;          // cell side >= largest tet bounding-box extent
    int nx, ny, nz;
};

// Error bits raised by device validation.
enum : unsigned { ERR_INDEX = 1u, ERR_VOLUME = 2u, ERR_REGION = 4u, ERR_HASH = 8u, ERR_FIXED = 16u, ERR_ROWBUF = 32u,
                  ERR_VEBUF = 64u };

// ---- launch wrappers (each returns the hipError_t of its launch) ----------
// scans / sorts (k_sort.hip)
size_t scan_temp_bytes(int64_t n);
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* temp,
                              hipStream_t s);  // out[n] = total (out has n+1 entries)
hipError_t exclusive_scan_u8_to_i32(const uint8_t* in, int32_t* out, int64_t n, void* temp,
                                    hipStream_t s);  // out[n] = total
size_t radix_sort_temp_bytes(int64_t n);
// Stable LSD radix sort of (key, value) on bits [0, nbits).  Result lands in
// keys/vals (buffers alt_* are scratch of the same size).
hipError_t radix_sort_u64_u32(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals,
                              int64_t n, int nbits, void* temp, hipStream_t s);
hipError_t reduce_max_i64(const int64_t* in, int64_t n, int64_t* out_dev, hipStream_t s);

// plan kernels (k_plan.hip)
struct MeshDev {
    const double* coords;   // [V][3]
    const int32_t* tets;    // [K][4]
    const uint8_t* vfree;   // [V]
    const uint8_t* region_in;  // optional
    int64_t V, K;
};
hipError_t launch_mesh_prep(const MeshDev& m, double* tetX, double* vol, uint8_t* region,
                            double* tet_min, double* ext_max_dev, double* bbox_dev,
                            unsigned* err, hipStream_t s);
hipError_t launch_free_ids(const uint8_t* vfree, const int32_t* scan, int64_t V, int32_t* free_id,
                           int32_t* free_to_vertex, hipStream_t s);
hipError_t launch_outer_flags(const uint8_t* region, const uint8_t* mask, int64_t K, int64_t* flags,
                              hipStream_t s);
hipError_t launch_outer_compact(const int64_t* flags, const int64_t* scan, int64_t K, int32_t* outer_ids,
                                hipStream_t s);
hipError_t launch_cell_keys(const double* tet_min, int64_t K, Grid g, uint64_t* keys, uint32_t* vals,
                            hipStream_t s);
hipError_t launch_cell_start(const uint64_t* sorted_keys, int64_t K, int64_t n_cells, int64_t* cell_start,
                             hipStream_t s);
// ball query: candidate count per outer tet (upper bound of its pairs), the
// tets' bounding boxes in cell order, then the classification of the
// candidates (the cand_n[oi] hits of each region compacted at its start,
// cand_code: one class byte per outer point; the hits counted per cut mask
// and per class), then the grouped compaction of the hits into the pair
// arrays.
hipError_t launch_cand_count(const double* tetX, const int32_t* outer_ids, int64_t n_outer,
                             const int64_t* cell_start, Grid g, double delta, int64_t* cand, hipStream_t s);
// (box: [K][2] float corners, sX: [K][12] vertex blocks, both in cell order)
hipError_t launch_sorted_boxes(const double* tetX, const uint32_t* cell_tets, int64_t K, float4* box, double* sX,
                               hipStream_t s);
// (cnt: [n_outer][16] hits per cut mask; cls: [n_outer][5] point-pair classes IN, CUT(0..3))
hipError_t launch_classify(const double* tetX, const int32_t* outer_ids, int64_t n_outer, const int64_t* cell_start,
                           const uint32_t* cell_tets, const float4* box, const double* sX, Grid g, double delta,
                           int strategy, const int64_t* cand_off, int64_t* cand_n, int64_t* cnt, uint32_t* cls,
                           int32_t* cand_m, uint32_t* cand_code, hipStream_t s);
hipError_t launch_pair_compact(int64_t n_outer, const int64_t* cand_off, const int64_t* cand_n, const int64_t* pair_off,
                               const int64_t* cnt, int strategy, const int32_t* cand_m, const uint32_t* cand_code,
                               int32_t* pair_m, uint16_t* pair_cls, hipStream_t s);
// pairs per outer tet into tot; class totals added to cls_tot[1..5] (zeroed by the caller)
hipError_t launch_pair_totals(const int64_t* cnt, const uint32_t* cls, int64_t n_outer, int64_t* tot,
                              unsigned long long* cls_tot, hipStream_t s);
// local vertex sets Ve of the outer tets: count pass writes ucount[oi] (and,
// given vbuf, the sorted sets there, vstride entries per outer tet, ERR_VEBUF
// for a longer set), fill pass writes the sorted sets at ve_off
hipError_t launch_pattern(bool fill, const int32_t* tets, int64_t n_outer, const int64_t* pair_off,
                          const int32_t* pair_m, int hash_cap, int64_t* ucount, const int64_t* ve_off, int32_t* ve_ids,
                          int32_t* vbuf, int vstride, unsigned* err, hipStream_t s);
// local vertex sets from the count pass's hand-off buffer (vstride entries per
// outer tet) to ve_ids at ve_off
hipError_t launch_ve_copy(int64_t n_outer, const int64_t* ve_off, const int32_t* vbuf, int vstride, int32_t* ve_ids,
                          hipStream_t s);

// numeric kernels (k_numeric.hip)
struct IntegrateArgs {
    const double* tetX;
    const double* vol;
    const uint8_t* region;
    const int32_t* tets;
    const int32_t* outer_ids;
    int64_t n_outer;
    const int64_t* pair_off;
    const int32_t* pair_m;
    const uint16_t* pair_cls;
    const int64_t* ve_off;
    const int32_t* ve_ids;
    const double* f_qp;  // may be null
    double delta, psi;
    int mc_samples;
    int caps;  // 1: cut points add the fullcaps Monte Carlo term (strategy fullcaps)
    int vr;    // 1: caps of cut pairs with n_in >= 1 sampled on E_m minus U_I (cone tets)
    int keying;  // 0: N samples per (outer point, element) pair; 1: N samples per element
    uint32_t key0, key1;
    int fx_shift;  // scale 2^fx_shift of the LDS sums T0 and R
    int g_shift;   // scale of the cut part of G_m (global accumulators)
    int w_shift;   // scale of the inside-count weight of G_m
    int umax;
    double* cblk;              // [sum |Ve|][4] cross blocks, at 4 * ve_off
    double* oblk;              // [n_outer][20]: 4x4 outer-outer block, then 4 load-vector terms
    unsigned long long* gacc;  // [22][gstride] two-word sums: 10 cut S2 sums, then the inside weight
    int64_t gstride;           // = K
    // R sums in global memory, [sum |Ve|][8] words (coarse k = 0..3, fine k = 0..3)
    // at 8 * (ve_off + i): for local vertex sets too large for LDS; nullptr: in LDS
    unsigned long long* rglob;
    // element keying: the per-plan sample table, row m at m * stab_stride
    // (stab_stride = sample_table_stride(N) words), or nullptr
    const unsigned long long* stab;
    int64_t stab_stride;
};
hipError_t launch_integrate(const IntegrateArgs& a, bool fp32, hipStream_t s);
// persistent: grid workgroups pull (mesh, outer position) items from a device
// queue (head reset by the launch); block 128 or 256
hipError_t launch_integrate_batch(const IntegrateArgs* descs, const int2* items, int64_t n_items,
                                  unsigned long long* head, int umax, bool fp32, bool vr, int keying, int block,
                                  int grid, hipStream_t s);
// one workgroup per work item (mesh, outer position), in list order; block 128 or 256
hipError_t launch_integrate_items(const IntegrateArgs* descs, const int2* items, int64_t n_items, int umax, bool fp32,
                                  bool vr, int keying, int block, hipStream_t s);
size_t integrate_lds_bytes(int umax);
// per-plan sample table of element keying: for every element m its N samples
// (counters (m, floor(s / 2), 0, 1)) packed one 64-bit word each, rows padded
// to a multiple of eight words plus one block of eight (read ahead by the
// sample loop)
inline int64_t sample_table_stride(int N) { return ((int64_t)N + 7) / 8 * 8 + 8; }
// (stride: the row length in words the caller allocated, at least
// sample_table_stride(N))
hipError_t launch_sample_table(int64_t K, int N, int64_t stride, uint32_t key0, uint32_t key1,
                               unsigned long long* tab, hipStream_t s);
// LDS of the integration with its R sums in global memory (independent of umax)
size_t integrate_global_lds_bytes();
// adds the exact-g defect of the T_Omega_I inner integrals to the load terms
// in oblk (tensor polynomial g of degree deg per axis, coefficients on the
// device; whole-element cap sampling only)
hipError_t launch_exact_g(const IntegrateArgs& a, const double* g_nodal, const double* coef, int deg, hipStream_t s);
// per-pair moments of outer positions [o_lo, o_hi): slot (p - pair_off[o_lo])*4 + k,
// out_S [slots][15], out_qm [slots][3] = (q, m, class)
hipError_t launch_debug_pairs(const IntegrateArgs& a, bool fp32, int64_t o_lo, int64_t o_hi, double* out_S,
                              int32_t* out_qm, hipStream_t s);
hipError_t launch_fill_zero_f64(double* p, int64_t n, hipStream_t s);
hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, int64_t n, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s);

// row-wise assembly (k_rows.hip)
struct RowPlan {
    const int32_t* tets;
    const uint8_t* region;
    const int32_t* inner_cnt;  // [K] pairs per inner tet (0: the tet occurs in no ball)
    const int32_t* free_id;
    const int32_t* free_to_vertex;
    const int32_t* outer_ids;
    const int32_t* outer_pos;  // [K] position among the outer tets or -1
    const int64_t* vt_off;     // [V+1] vertex -> (4 tet + local index), sorted by tet
    const uint32_t* vt_val;
    const int64_t* ve_off;
    const int32_t* ve_ids;
    const int32_t* ve_owner;   // [sum |Ve|] outer position owning each entry
    const int64_t* inc_off;    // [V+1] vertex -> entries of the Ve sets holding it
    const uint32_t* inc_val;
    const int64_t* ff_row_ptr;
    const int64_t* fc_row_ptr;
    const int32_t* all_cols;   // sorted vertex columns of each row, at ff_row_ptr[r] + fc_row_ptr[r]
    const int32_t* fc_col;
    int max_row;
};
struct RowNumeric {
    const double* cblk;
    const double* oblk;
    const double* gvals;  // [K][10] G_m upper triangles
    const double* g_nodal;
    int row_shift;
    double* ff_val;
    double* fc_val;
    double* rhs;
};
hipError_t launch_vt_keys(const int32_t* tets, int64_t K, uint64_t* keys, uint32_t* vals, hipStream_t s);
// off[k] = first position of sorted key >= k, for k in [0, n_keys]
hipError_t launch_offsets(const uint64_t* skeys, int64_t n, int64_t n_keys, int64_t* off, hipStream_t s);
hipError_t launch_inc_keys(const int64_t* ve_off, int64_t n_outer, const int32_t* ve_ids, uint64_t* keys,
                           uint32_t* vals, int32_t* owner, hipStream_t s);
hipError_t launch_inner_count(const int64_t* pair_off, int64_t n_outer, const int32_t* pair_m, int32_t* inner_cnt,
                              hipStream_t s);
hipError_t launch_outer_pos(const int32_t* outer_ids, int64_t n_outer, int32_t* outer_pos, int64_t K, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// CSR pattern, count pass (fill = false: n_ff / n_fc per row, the columns
// left unordered in rowbuf [n_rows][hash_cap]) then fill pass (fill = true,
// the same rowbuf and counts)
hipError_t launch_row_pattern(bool fill, const RowPlan& rp, int64_t n_rows, int hash_cap, int row_stride, int64_t* n_ff,
                              int64_t* n_fc, const int64_t* ff_row_ptr, const int64_t* fc_row_ptr, int32_t* all_cols,
                              int32_t* ff_col, int32_t* fc_col, uint32_t* rowbuf, unsigned* err, hipStream_t s);
hipError_t launch_g_finalize(int64_t K, const uint8_t* region, const int32_t* inner_cnt, const double* vol,
                             const unsigned long long* gacc, int g_shift, int w_shift, double* gvals, hipStream_t s);
size_t row_assemble_lds_bytes(int max_row);  // dynamic part
// rows too long for LDS: their three-word sums in global memory, 3 words per
// nonzero of the row at 3 * (ff_row_ptr[r] + fc_row_ptr[r]) (racc), the
// columns read from all_cols
hipError_t launch_row_assemble_global(const RowPlan& rp, const RowNumeric& nm, unsigned long long* racc,
                                      int64_t n_rows, hipStream_t s);
size_t row_assemble_static_lds();
hipError_t launch_row_assemble(const RowPlan& rp, const RowNumeric& nm, int64_t n_rows, hipStream_t s);

// CG (k_cg.hip)
// Device-side state of one CG solve.  The first 32 bytes are what the host
// polls.
struct CgState {
    int iter, done, max_iter, pad;  // done: 0 running, 1 converged, 2 breakdown, 3 cap, 4 b = 0
    double res2, bnorm;             // latest ||r||^2, ||b||
    double rr[2];                   // ||r_i||^2 at iteration parity i & 1
    double pAp, bb, thr;
};
constexpr size_t kCgPollBytes = 32;
// largest n of the allocation-free CG (its static device scratch holds 3 n doubles)
constexpr int64_t kCgNoAllocMaxN = (int64_t)1 << 19;
constexpr int kMaxDevices = 64;
size_t cg_work_doubles(int64_t n);  // r, p, Ap, dot partials, state
hipError_t launch_spmv(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* x,
                       double* y, hipStream_t s);
// r = b - A x, p = r, ||r||^2, ||b||^2, threshold and the initial decision
hipError_t cg_enqueue_start(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, const double* b,
                            double* x, double rtol, int max_iter, double* work, hipStream_t s);
// iterations it0 .. it0 + count - 1 (no-ops once the state says stop)
hipError_t cg_enqueue_iterations(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, double* x,
                                 int it0, int count, double* work, hipStream_t s);
hipError_t cg_enqueue_zero(int64_t n, double* x, hipStream_t s);
const CgState* cg_state(const double* work, int64_t n);  // device address of the state in work
// the allocation-free CG's scratch on `device` (the current device): resolved
// once per device with hipGetSymbolAddress
hipError_t cg_noalloc_setup(int device, void** out);
void* cg_noalloc_scratch(int device);  // nullptr before setup

}  // namespace nlfem
