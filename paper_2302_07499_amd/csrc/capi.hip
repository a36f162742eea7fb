// Host runtime behind the C ABI of include/nlfem.h: contexts, the symbolic
// plan (mesh layout, cell list, classification, local vertex sets,
// vertex-keyed sorted lists, CSR pattern), the numeric assembly, batches and
// the CG solver loop.  Device memory management is in runtime.hip, the
// request server in server.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <atomic>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "runtime.hpp"

using namespace nlfem;

namespace {

int bits_for(uint64_t x) {  // number of bits needed to represent values in [0, x]
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct nlfem_plan {
    nlfem_ctx* ctx = nullptr;
    std::vector<void*> owned;
    // sizes
    int64_t V = 0, K = 0, n_free = 0, n_outer = 0, P = 0, ve_total = 0;
    int64_t nnz_ff = 0, nnz_fc = 0, max_pairs = 0, max_inner = 0, max_vt = 0;
    int umax = 0, max_row = 0, fx_shift = 0, g_shift = 0, w_shift = 0, row_shift = 0;
    int64_t pair_counts[5] = {0, 0, 0, 0, 0};
    double delta = 0, psi = 0;
    int mc = 1, precision = 0, strategy = 0, cap_sampling = 0, keying = 0;
    uint64_t seed = 0;
    // device arrays: mesh and ball query
    double *tetX = nullptr, *vol = nullptr;
    int32_t* tets = nullptr;
    uint8_t* region = nullptr;
    int32_t *free_id = nullptr, *free_to_vertex = nullptr, *outer_ids = nullptr, *outer_pos = nullptr;
    int64_t* pair_off = nullptr;
    int32_t* pair_m = nullptr;
    uint16_t* pair_cls = nullptr;
    int32_t* inner_cnt = nullptr;
    // local vertex sets and the vertex-keyed lists
    int64_t *ve_off = nullptr, *vt_off = nullptr, *inc_off = nullptr;
    int32_t *ve_ids = nullptr, *ve_owner = nullptr;
    uint32_t *vt_val = nullptr, *inc_val = nullptr;
    // CSR pattern
    int64_t *ff_row_ptr = nullptr, *fc_row_ptr = nullptr;
    int32_t *ff_col = nullptr, *fc_col = nullptr, *all_cols = nullptr;
    // numeric workspace
    double *cblk = nullptr, *oblk = nullptr, *gvals = nullptr, *fc_val_int = nullptr;
    unsigned long long* gacc = nullptr;
    // sums in global memory where LDS is too small (else nullptr)
    bool global_r = false, global_rows = false;
    unsigned long long* rglob = nullptr;  // [ve_total][8] R words of the integration
    unsigned long long* racc = nullptr;   // [3 (nnz_ff + nnz_fc)] row sums
    unsigned long long* stab = nullptr;   // element keying: [K][stab_stride] samples
    int64_t stab_stride = 0;
    double times[6] = {0, 0, 0, 0, 0, 0};

    template <typename Tp>
    Tp* alloc(size_t n) {
        void* p = dalloc(ctx, n * sizeof(Tp));
        if (p) owned.push_back(p);
        return (Tp*)p;
    }
    void release() {
        for (void* p : owned) dfree(ctx, p);
        owned.clear();
    }
};

namespace {

// threads that build the plans of a batch (each with its own stream)
constexpr int kBuilders = 4;

// scoped temporary device buffer
struct Tmp {
    nlfem_ctx* c;
    void* p = nullptr;
    Tmp(nlfem_ctx* c_, size_t bytes) : c(c_) { p = dalloc(c, bytes); }
    ~Tmp() { dfree(c, p); }
    template <typename Tp>
    Tp* as() {
        return (Tp*)p;
    }
};

struct Timer {
    hipEvent_t a, b;
    hipStream_t s;
    explicit Timer(hipStream_t s_) : s(s_) {
        hipEventCreate(&a);
        hipEventCreate(&b);
        hipEventRecord(a, s);
    }
    double stop() {
        hipEventRecord(b, s);
        hipEventSynchronize(b);
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        hipEventDestroy(a);
        hipEventDestroy(b);
    }
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            return fail(c, NLFEM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                                         \
    } while (0)

// plan memory comes from the plan's context (pl->ctx), temporaries (TMP) and
// the stream from the context c that builds it (the same one unless a batch
// builds its plans on several threads)
#define ALLOC(ptr, T, n)                                      \
    do {                                                      \
        ptr = pl->alloc<T>((size_t)(n));                      \
        if (!ptr) return fail(c, NLFEM_E_OOM, owner_err(pl));  \
    } while (0)

#define TMP(name, bytes)                                       \
    Tmp name(c, (bytes));                                      \
    if (!name.p) return fail(c, NLFEM_E_OOM, c->err)

std::string owner_err(nlfem_plan* pl) {
    std::lock_guard<std::recursive_mutex> lk(pl->ctx->mu);
    return pl->ctx->err;
}

int64_t read_i64(nlfem_ctx* c, const int64_t* dev) {
    hipMemcpyAsync(c->pinned_i, dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    drain_pending(c);
    return c->pinned_i[0];
}

RowPlan make_row_plan(nlfem_plan* pl);

// shift s with bound * 2^s < 2^62
int shift_for(double bound) {
    if (!(bound > 0.0) || !std::isfinite(bound)) return 62;
    int e = 0;
    std::frexp(bound, &e);  // bound < 2^e
    return std::min(62 - e, 1000);
}

// element keying without the cap region reads its samples from a per-plan
// table (K sample_table_stride(N) words) instead of drawing them per pair
bool uses_sample_table(const nlfem_plan* pl) {
    return pl->keying == NLFEM_KEY_ELEMENT && pl->strategy == NLFEM_FULLCAPS &&
           pl->cap_sampling != NLFEM_CAPS_OUTSIDE_UI && pl->mc > 0;
}

nlfem_status build_plan(nlfem_ctx* c, nlfem_plan* pl, const nlfem_mesh* mesh, const nlfem_params* prm) {
    hipStream_t s = c->stream;
    const int64_t V = mesh->n_vertices, K = mesh->n_tets;
    pl->V = V;
    pl->K = K;
    Timer total(s);
    // ---- mesh on device -------------------------------------------------
    const double* coords = mesh->coords;
    const int32_t* tets = mesh->tets;
    const uint8_t* vfree = mesh->vertex_free;
    const uint8_t* region_in = mesh->tet_region;
    const uint8_t* mask = prm->outer_mask;
    Tmp t_coords(c, mesh->mem_kind == 0 ? (size_t)V * 24 + 8 : 8);
    Tmp t_vfree(c, mesh->mem_kind == 0 ? (size_t)V + 8 : 8);
    Tmp t_region(c, (mesh->mem_kind == 0 && region_in) ? (size_t)K + 8 : 8);
    Tmp t_mask(c, (mesh->mem_kind == 0 && mask) ? (size_t)K + 8 : 8);
    if (!t_coords.p || !t_vfree.p || !t_region.p || !t_mask.p) return fail(c, NLFEM_E_OOM, c->err);
    ALLOC(pl->tets, int32_t, 4 * K + 4);
    if (mesh->mem_kind == 0) {
        if (V) HIPCHK(hipMemcpyAsync(t_coords.p, coords, (size_t)V * 24, hipMemcpyHostToDevice, s));
        if (V) HIPCHK(hipMemcpyAsync(t_vfree.p, vfree, (size_t)V, hipMemcpyHostToDevice, s));
        if (K) HIPCHK(hipMemcpyAsync(pl->tets, tets, (size_t)K * 16, hipMemcpyHostToDevice, s));
        if (region_in && K) HIPCHK(hipMemcpyAsync(t_region.p, region_in, (size_t)K, hipMemcpyHostToDevice, s));
        if (mask && K) HIPCHK(hipMemcpyAsync(t_mask.p, mask, (size_t)K, hipMemcpyHostToDevice, s));
        coords = t_coords.as<double>();
        vfree = t_vfree.as<uint8_t>();
        if (region_in) region_in = t_region.as<uint8_t>();
        if (mask) mask = t_mask.as<uint8_t>();
    } else {
        if (K) HIPCHK(hipMemcpyAsync(pl->tets, tets, (size_t)K * 16, hipMemcpyDeviceToDevice, s));
    }
    ALLOC(pl->tetX, double, 12 * K + 12);
    ALLOC(pl->vol, double, K + 1);
    ALLOC(pl->region, uint8_t, K + 8);
    TMP(t_min, (size_t)3 * K * 8 + 8);
    TMP(t_small, 32 * sizeof(double));
    TMP(t_err, 64);
    HIPCHK(hipMemsetAsync(t_err.p, 0, 64, s));
    MeshDev md{coords, pl->tets, vfree, region_in, V, K};
    double* small = t_small.as<double>();
    HIPCHK(launch_mesh_prep(md, pl->tetX, pl->vol, pl->region, t_min.as<double>(), small, small + 1,
                            t_err.as<unsigned>(), s));
    // free ids
    ALLOC(pl->free_id, int32_t, V + 1);
    TMP(t_fscan, (size_t)(V + 2) * 4);
    TMP(t_scantmp, (size_t)(2 * V + 8) * 8 + scan_temp_bytes(V + 1) + scan_temp_bytes(K + 1) + 4096);
    HIPCHK(exclusive_scan_u8_to_i32(vfree, t_fscan.as<int32_t>(), V, t_scantmp.p, s));
    int32_t nf32 = 0;
    HIPCHK(hipMemcpyAsync(&nf32, t_fscan.as<int32_t>() + V, 4, hipMemcpyDeviceToHost, s));
    unsigned errbits = 0;
    HIPCHK(hipMemcpyAsync(&errbits, t_err.p, 4, hipMemcpyDeviceToHost, s));
    double hs_small[8];
    HIPCHK(hipMemcpyAsync(hs_small, small, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (errbits & ERR_INDEX) return fail(c, NLFEM_E_MESH, "tet vertex index out of range");
    if (errbits & ERR_VOLUME) return fail(c, NLFEM_E_MESH, "zero-volume tetrahedron");
    if (errbits & ERR_REGION) return fail(c, NLFEM_E_MESH, "free vertex in a tet marked as T_OmegaI");
    pl->n_free = nf32;
    const int64_t nf = pl->n_free;
    ALLOC(pl->free_to_vertex, int32_t, nf + 1);
    HIPCHK(launch_free_ids(vfree, t_fscan.as<int32_t>(), V, pl->free_id, pl->free_to_vertex, s));
    // outer tets
    TMP(t_oflags, (size_t)(K + 1) * 8);
    TMP(t_oscan, (size_t)(K + 2) * 8);
    HIPCHK(launch_outer_flags(pl->region, mask, K, t_oflags.as<int64_t>(), s));
    HIPCHK(exclusive_scan_i64(t_oflags.as<int64_t>(), t_oscan.as<int64_t>(), K, t_scantmp.p, s));
    pl->n_outer = read_i64(c, t_oscan.as<int64_t>() + K);
    const int64_t no = pl->n_outer;
    ALLOC(pl->outer_ids, int32_t, no + 1);
    HIPCHK(launch_outer_compact(t_oflags.as<int64_t>(), t_oscan.as<int64_t>(), K, pl->outer_ids, s));
    // ---- cell list --------------------------------------------------------
    const double ext = hs_small[0];
    Grid g;
    double cs = ext > 0 ? ext * (1.0 + 1e-12) : 1.0;
    double bmin[3] = {hs_small[1], hs_small[2], hs_small[3]}, bmax[3] = {hs_small[4], hs_small[5], hs_small[6]};
    int dims[3];
    while (true) {
        double cells = 1;
        for (int i = 0; i < 3; ++i) {
            dims[i] = (int)std::floor((bmax[i] - bmin[i]) / cs) + 1;
            if (dims[i] < 1) dims[i] = 1;
            cells *= dims[i];
        }
        if (cells <= (double)(1 << 24)) break;
        cs *= 1.25;
    }
    g.ox = bmin[0]; g.oy = bmin[1]; g.oz = bmin[2];
    g.cs = cs;
    g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
    const int64_t n_cells = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t* cell_start = nullptr;
    uint32_t* cell_tets = nullptr;
    TMP(t_cstart, (size_t)(n_cells + 2) * 8);
    TMP(t_ckeys, (size_t)(K + 1) * 8 * 2);
    TMP(t_cvals, (size_t)(K + 1) * 4 * 2);
    TMP(t_rstmp, radix_sort_temp_bytes(K + 1));
    cell_start = t_cstart.as<int64_t>();
    {
        uint64_t* keys = t_ckeys.as<uint64_t>();
        uint32_t* vals = t_cvals.as<uint32_t>();
        HIPCHK(launch_cell_keys(t_min.as<double>(), K, g, keys, vals, s));
        HIPCHK(radix_sort_u64_u32(keys, vals, keys + K, vals + K, K, bits_for((uint64_t)n_cells), t_rstmp.p, s));
        HIPCHK(launch_cell_start(keys, K, n_cells, cell_start, s));
        cell_tets = vals;
    }
    // ---- classification -------------------------------------------------
    Timer tcls(s);
    TMP(t_cnt, (size_t)(16 * no + 16) * 8);
    TMP(t_cls, (size_t)(5 * no + 5) * 4);
    TMP(t_cc, 64);
    TMP(t_tot, (size_t)(no + 1) * 8);
    TMP(t_cand_off, (size_t)(no + 2) * 8);
    ALLOC(pl->pair_off, int64_t, no + 2);
    TMP(t_scan2, scan_temp_bytes(no + 1) + scan_temp_bytes(K + 1) + 4096);
    HIPCHK(launch_cand_count(pl->tetX, pl->outer_ids, no, cell_start, g, prm->delta, t_tot.as<int64_t>(), s));
    HIPCHK(exclusive_scan_i64(t_tot.as<int64_t>(), t_cand_off.as<int64_t>(), no, t_scan2.p, s));
    const int64_t n_cand = read_i64(c, t_cand_off.as<int64_t>() + no);
    TMP(t_cand_m, (size_t)(n_cand + 1) * 4);
    TMP(t_cand_c, (size_t)(n_cand + 1) * 4);
    TMP(t_cand_n, (size_t)(no + 1) * 8);
    TMP(t_box, (size_t)(K + 1) * 32);
    TMP(t_sx, (size_t)(K + 1) * 96);
    HIPCHK(launch_sorted_boxes(pl->tetX, cell_tets, K, (float4*)t_box.p, t_sx.as<double>(), s));
    HIPCHK(launch_classify(pl->tetX, pl->outer_ids, no, cell_start, cell_tets, (const float4*)t_box.p,
                           t_sx.as<double>(), g, prm->delta, prm->strategy, t_cand_off.as<int64_t>(),
                           t_cand_n.as<int64_t>(), t_cnt.as<int64_t>(), t_cls.as<uint32_t>(),
                           t_cand_m.as<int32_t>(), t_cand_c.as<uint32_t>(), s));
    HIPCHK(hipMemsetAsync(t_cc.p, 0, 64, s));
    HIPCHK(launch_pair_totals(t_cnt.as<int64_t>(), t_cls.as<uint32_t>(), no, t_tot.as<int64_t>(),
                              t_cc.as<unsigned long long>(), s));
    HIPCHK(exclusive_scan_i64(t_tot.as<int64_t>(), pl->pair_off, no, t_scan2.p, s));
    HIPCHK(reduce_max_i64(t_tot.as<int64_t>(), no, (int64_t*)(small + 8), s));
    pl->P = read_i64(c, pl->pair_off + no);
    pl->max_pairs = read_i64(c, (int64_t*)(small + 8));
    const int64_t P = pl->P;
    if (P >= (int64_t)0xFFFFFFFFll) return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^32 pairs in one plan");
    // the fine fixed-point words take < 2^48 per contribution and must not overflow 2^63
    if (pl->max_pairs >= ((int64_t)1 << 15))
        return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^15 interacting tets for one outer tet");
    ALLOC(pl->pair_m, int32_t, P + 1);
    ALLOC(pl->pair_cls, uint16_t, P + 1);
    HIPCHK(launch_pair_compact(no, t_cand_off.as<int64_t>(), t_cand_n.as<int64_t>(), pl->pair_off,
                               t_cnt.as<int64_t>(), prm->strategy, t_cand_m.as<int32_t>(), t_cand_c.as<uint32_t>(),
                               pl->pair_m, pl->pair_cls, s));
    {
        unsigned long long cc[6];
        HIPCHK(hipMemcpyAsync(cc, t_cc.p, sizeof cc, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < 5; ++i) pl->pair_counts[i] = (int64_t)cc[1 + i];
    }
    pl->times[1] = tcls.stop();
    Timer tpat(s);
    // ---- pairs per inner tet, outer positions ----------------------------
    ALLOC(pl->inner_cnt, int32_t, K + 1);
    ALLOC(pl->outer_pos, int32_t, K + 1);
    HIPCHK(launch_fill_i32(pl->inner_cnt, K, 0, s));
    HIPCHK(launch_inner_count(pl->pair_off, no, pl->pair_m, pl->inner_cnt, s));
    HIPCHK(launch_outer_pos(pl->outer_ids, no, pl->outer_pos, K, s));
    {
        std::vector<int32_t> ic(K);
        if (K) HIPCHK(hipMemcpyAsync(ic.data(), pl->inner_cnt, (size_t)K * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int64_t e = 0; e < K; ++e) pl->max_inner = std::max<int64_t>(pl->max_inner, ic[e]);
    }
    if (pl->max_inner >= ((int64_t)1 << 15))
        return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^15 outer tets interacting with one inner tet");
    // ---- local vertex sets ---------------------------------------------------
    TMP(t_ucount, (size_t)(no + 1) * 8);
    int hash_cap = (int)std::max<int64_t>(256, next_pow2(2 * (pl->max_pairs + 16)));
    // the count pass leaves each set in a hand-off buffer of vstride entries
    // per outer tet (a set holds fewer vertices than half its outer tet's
    // pairs on the measured workloads), if that takes at most 2 GiB; a longer
    // set, or no buffer, leaves the sets to the fill pass.  NLFEM_VE_STRIDE
    // (a power of two, for checks) sets the stride.
    int vstride = (int)next_pow2(std::max<int64_t>(64, (pl->max_pairs + 1) / 2));
    if (const char* vs = std::getenv("NLFEM_VE_STRIDE")) {
        const long v = std::strtol(vs, nullptr, 10);
        if (v >= 1 && v <= (1 << 24) && (v & (v - 1)) == 0) vstride = (int)v;
    }
    std::unique_ptr<Tmp> t_vbuf;
    if ((size_t)std::max<int64_t>(no, 1) * (size_t)vstride * 4 <= ((size_t)2 << 30)) {
        t_vbuf.reset(new Tmp(c, (size_t)std::max<int64_t>(no, 1) * (size_t)vstride * 4));
        if (!t_vbuf->p) t_vbuf.reset();  // no room: the fill pass builds the sets
    }
    while (true) {
        if ((size_t)hash_cap * 4 > c->lds_max)
            return fail(c, NLFEM_E_UNSUPPORTED, "local vertex set too large for LDS");
        HIPCHK(launch_fill_i32((int32_t*)t_err.p, 16, 0, s));
        HIPCHK(launch_pattern(false, pl->tets, no, pl->pair_off, pl->pair_m, hash_cap, t_ucount.as<int64_t>(), nullptr,
                              nullptr, t_vbuf ? t_vbuf->as<int32_t>() : nullptr, vstride, t_err.as<unsigned>(), s));
        HIPCHK(hipMemcpyAsync(&errbits, t_err.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!(errbits & ERR_HASH)) break;
        hash_cap *= 2;
    }
    const bool ve_handoff = t_vbuf && !(errbits & ERR_VEBUF);
    ALLOC(pl->ve_off, int64_t, no + 2);
    HIPCHK(exclusive_scan_i64(t_ucount.as<int64_t>(), pl->ve_off, no, t_scan2.p, s));
    HIPCHK(reduce_max_i64(t_ucount.as<int64_t>(), no, (int64_t*)(small + 8), s));
    pl->umax = (int)read_i64(c, (int64_t*)(small + 8));
    pl->ve_total = read_i64(c, pl->ve_off + no);
    const int64_t VT = pl->ve_total;
    // local vertex sets beyond LDS: the integration keeps its R sums in global memory
    // (NLFEM_GLOBAL_SUMS=1 in the environment forces both global forms, for checks)
    const char* force_global = std::getenv("NLFEM_GLOBAL_SUMS");
    const bool force = force_global && force_global[0] == '1';
    pl->global_r = force || integrate_lds_bytes(pl->umax) > c->lds_max;
    if (pl->global_r && (pl->umax >= 65536 || integrate_global_lds_bytes() > c->lds_max))
        return fail(c, NLFEM_E_UNSUPPORTED, "ball vertex set of one outer tet beyond 65535 vertices");
    if (VT >= (int64_t)0xFFFFFFFFll || 4 * K >= (int64_t)0xFFFFFFFFll)
        return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^32 local vertex set entries");
    ALLOC(pl->ve_ids, int32_t, VT + 1);
    if (ve_handoff)
        HIPCHK(launch_ve_copy(no, pl->ve_off, t_vbuf->as<int32_t>(), vstride, pl->ve_ids, s));
    else
        HIPCHK(launch_pattern(true, pl->tets, no, pl->pair_off, pl->pair_m, hash_cap, t_ucount.as<int64_t>(),
                              pl->ve_off, pl->ve_ids, nullptr, 0, t_err.as<unsigned>(), s));
    t_vbuf.reset();
    // ---- vertex -> tets and vertex -> local vertex set entries -------------
    ALLOC(pl->vt_off, int64_t, V + 2);
    ALLOC(pl->vt_val, uint32_t, 4 * K + 1);
    ALLOC(pl->inc_off, int64_t, V + 2);
    ALLOC(pl->inc_val, uint32_t, VT + 1);
    ALLOC(pl->ve_owner, int32_t, VT + 1);
    const int vbits = std::max(1, bits_for((uint64_t)V));
    {
        TMP(t_k, (size_t)(4 * K + 1) * 16);
        TMP(t_v, (size_t)(4 * K + 1) * 8);
        TMP(t_rs, radix_sort_temp_bytes(4 * K + 1));
        uint64_t* keys = t_k.as<uint64_t>();
        uint32_t* vals = t_v.as<uint32_t>();
        HIPCHK(launch_vt_keys(pl->tets, K, keys, vals, s));
        HIPCHK(radix_sort_u64_u32(keys, vals, keys + 4 * K, vals + 4 * K, 4 * K, vbits, t_rs.p, s));
        HIPCHK(launch_offsets(keys, 4 * K, V, pl->vt_off, s));
        HIPCHK(launch_copy_i32((const int32_t*)vals, (int32_t*)pl->vt_val, 4 * K, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    {
        TMP(t_k, (size_t)(VT + 1) * 16);
        TMP(t_v, (size_t)(VT + 1) * 8);
        TMP(t_rs, radix_sort_temp_bytes(VT + 1));
        uint64_t* keys = t_k.as<uint64_t>();
        uint32_t* vals = t_v.as<uint32_t>();
        HIPCHK(launch_inc_keys(pl->ve_off, no, pl->ve_ids, keys, vals, pl->ve_owner, s));
        HIPCHK(radix_sort_u64_u32(keys, vals, keys + VT, vals + VT, VT, vbits, t_rs.p, s));
        HIPCHK(launch_offsets(keys, VT, V, pl->inc_off, s));
        HIPCHK(launch_copy_i32((const int32_t*)vals, (int32_t*)pl->inc_val, VT, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    {
        std::vector<int64_t> vo(V + 1);
        HIPCHK(hipMemcpyAsync(vo.data(), pl->vt_off, (size_t)(V + 1) * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int64_t v = 0; v < V; ++v) pl->max_vt = std::max<int64_t>(pl->max_vt, vo[v + 1] - vo[v]);
    }
    // the fine words of a row slot take < 2^48 from each of at most 4 max_vt terms
    if (pl->max_vt >= ((int64_t)1 << 13)) return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^13 tets at one vertex");
    // ---- CSR pattern, row by row -------------------------------------------
    RowPlan rp = make_row_plan(pl);
    TMP(t_nff, (size_t)(nf + 2) * 8);
    TMP(t_nfc, (size_t)(nf + 2) * 8);
    // hash capacity per row (4 |Ve| slots at least), and the row buffer's
    // stride: half the hash set first (the widest rows hold somewhat more
    // than |Ve| columns), doubled (the count pass run again) if a row does
    // not fit
    int row_cap = (int)std::max<int64_t>(512, next_pow2(4 * (int64_t)std::max(pl->umax, 1)));
    int row_stride = row_cap / 2;
    // NLFEM_ROW_STRIDE=<words> (a power of two, for checks) starts narrower, so
    // that the overflow retry runs
    if (const char* rs = std::getenv("NLFEM_ROW_STRIDE")) {
        const long v = std::strtol(rs, nullptr, 10);
        if (v >= 1 && v <= row_cap / 2 && (v & (v - 1)) == 0) row_stride = (int)v;
    }
    std::unique_ptr<Tmp> t_rows;  // [nf][row_stride] each row's columns between the two passes
    while (true) {
        if ((size_t)row_cap * 4 + 2048 > c->lds_max) return fail(c, NLFEM_E_UNSUPPORTED, "matrix row too large for LDS");
        t_rows.reset();
        t_rows.reset(new Tmp(c, (size_t)std::max<int64_t>(nf, 1) * (size_t)row_stride * 4));
        if (!t_rows->p) return fail(c, NLFEM_E_OOM, c->err);
        HIPCHK(launch_fill_i32((int32_t*)t_err.p, 16, 0, s));
        HIPCHK(launch_row_pattern(false, rp, nf, row_cap, row_stride, t_nff.as<int64_t>(), t_nfc.as<int64_t>(), nullptr,
                                  nullptr, nullptr, nullptr, nullptr, t_rows->as<uint32_t>(), t_err.as<unsigned>(), s));
        HIPCHK(hipMemcpyAsync(&errbits, t_err.p, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (errbits & ERR_HASH) {
            row_cap *= 2;
            row_stride = std::max(row_stride, row_cap / 2);
        } else if (errbits & ERR_ROWBUF) {
            row_stride *= 2;  // at most row_cap: a row never holds more columns than its hash set
        } else {
            break;
        }
    }
    ALLOC(pl->ff_row_ptr, int64_t, nf + 2);
    ALLOC(pl->fc_row_ptr, int64_t, nf + 2);
    HIPCHK(exclusive_scan_i64(t_nff.as<int64_t>(), pl->ff_row_ptr, nf, t_scan2.p, s));
    HIPCHK(exclusive_scan_i64(t_nfc.as<int64_t>(), pl->fc_row_ptr, nf, t_scan2.p, s));
    pl->nnz_ff = read_i64(c, pl->ff_row_ptr + nf);
    pl->nnz_fc = read_i64(c, pl->fc_row_ptr + nf);
    {
        std::vector<int64_t> a(nf), b(nf);
        if (nf) {
            HIPCHK(hipMemcpyAsync(a.data(), t_nff.p, (size_t)nf * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(b.data(), t_nfc.p, (size_t)nf * 8, hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        for (int64_t r = 0; r < nf; ++r) pl->max_row = (int)std::max<int64_t>(pl->max_row, a[r] + b[r]);
    }
    // rows beyond LDS: the row assembly keeps its sums in global memory
    pl->global_rows = force || row_assemble_lds_bytes(pl->max_row) + row_assemble_static_lds() > c->lds_max;
    ALLOC(pl->ff_col, int32_t, pl->nnz_ff + 1);
    ALLOC(pl->fc_col, int32_t, pl->nnz_fc + 1);
    ALLOC(pl->all_cols, int32_t, pl->nnz_ff + pl->nnz_fc + 1);
    HIPCHK(launch_row_pattern(true, rp, nf, row_cap, row_stride, t_nff.as<int64_t>(), t_nfc.as<int64_t>(), pl->ff_row_ptr,
                              pl->fc_row_ptr, pl->all_cols, pl->ff_col, pl->fc_col, t_rows->as<uint32_t>(),
                              t_err.as<unsigned>(), s));
    HIPCHK(hipStreamSynchronize(s));
    t_rows.reset();
    pl->times[2] = tpat.stop();
    // ---- numeric workspace -------------------------------------------------
    ALLOC(pl->cblk, double, 4 * VT + 4);
    ALLOC(pl->oblk, double, 20 * no + 20);
    ALLOC(pl->gacc, unsigned long long, 22 * K + 22);
    ALLOC(pl->gvals, double, 10 * K + 10);
    ALLOC(pl->fc_val_int, double, pl->nnz_fc + 1);
    if (pl->global_r) ALLOC(pl->rglob, unsigned long long, 8 * VT + 8);
    if (pl->global_rows) ALLOC(pl->racc, unsigned long long, 3 * (pl->nnz_ff + pl->nnz_fc) + 3);
    if (uses_sample_table(pl)) {
        pl->stab_stride = sample_table_stride(pl->mc);
        ALLOC(pl->stab, unsigned long long, K * pl->stab_stride + 8);
        HIPCHK(launch_sample_table(K, pl->mc, pl->stab_stride, (uint32_t)(pl->seed & 0xFFFFFFFFull),
                                   (uint32_t)(pl->seed >> 32), pl->stab, s));
    }
    // fixed-point scales (each sum stays below 2^62 in units of its coarse word):
    //  T0_k, R_k(v) <= B_R = sum over the pair list of f_m S0 <= 4 max_pairs max|E|
    //    (S0 <= 2 |E_m| for one pair: subtets plus a Monte Carlo count of at most N)
    //  G_m cut part <= |psi| max|E|^2 2 max_inner, inside weight <= |psi| max|E| max_inner
    //  one row slot: at most 4 max_vt terms of C, O (<= |psi| max|E| B_R / 4) or G
    {
        TMP(t_vmax, 16);
        HIPCHK(reduce_max_i64((const int64_t*)pl->vol, K, t_vmax.as<int64_t>(), s));  // non-negative doubles
        int64_t bitsv = read_i64(c, t_vmax.as<int64_t>());
        double vmax;
        std::memcpy(&vmax, &bitsv, 8);
        const double apsi = std::fabs(pl->psi);
        const double bR = 4.0 * (double)std::max<int64_t>(pl->max_pairs, 1) * vmax;
        const double bW = 2.0 * apsi * vmax * (double)std::max<int64_t>(pl->max_inner, 1);
        const double bG = 4.0 * apsi * vmax * vmax * (double)std::max<int64_t>(pl->max_inner, 1);
        const double bC = apsi * vmax * bR * 0.5 + bG + bW * vmax;
        const double bRow = bC * 8.0 * (double)std::max<int64_t>(pl->max_vt, 1);
        // a single term must also stay below 2^51 units (the integer split of
        // the integration kernel): at most 4 max|E| for T0 and R, |psi| max|E|
        // for the inside weight, 2 |psi| max|E|^2 for the cut part of G_m
        pl->fx_shift = std::min(shift_for(bR), shift_for(4.0 * vmax * 2048.0));
        pl->w_shift = std::min(shift_for(bW), shift_for(apsi * vmax * 2048.0));
        pl->g_shift = std::min(shift_for(bG), shift_for(2.0 * apsi * vmax * vmax * 2048.0));
        pl->row_shift = shift_for(bRow);
    }
    pl->times[0] = total.stop();
    return NLFEM_OK;
}

RowPlan make_row_plan(nlfem_plan* pl) {
    RowPlan rp;
    rp.tets = pl->tets;
    rp.region = pl->region;
    rp.inner_cnt = pl->inner_cnt;
    rp.free_id = pl->free_id;
    rp.free_to_vertex = pl->free_to_vertex;
    rp.outer_ids = pl->outer_ids;
    rp.outer_pos = pl->outer_pos;
    rp.vt_off = pl->vt_off;
    rp.vt_val = pl->vt_val;
    rp.ve_off = pl->ve_off;
    rp.ve_ids = pl->ve_ids;
    rp.ve_owner = pl->ve_owner;
    rp.inc_off = pl->inc_off;
    rp.inc_val = pl->inc_val;
    rp.ff_row_ptr = pl->ff_row_ptr;
    rp.fc_row_ptr = pl->fc_row_ptr;
    rp.all_cols = pl->all_cols;
    rp.fc_col = pl->fc_col;
    rp.max_row = std::max(pl->max_row, 1);
    return rp;
}

IntegrateArgs make_args(nlfem_plan* pl, const double* f_qp) {
    IntegrateArgs a;
    a.tetX = pl->tetX;
    a.vol = pl->vol;
    a.region = pl->region;
    a.tets = pl->tets;
    a.outer_ids = pl->outer_ids;
    a.n_outer = pl->n_outer;
    a.pair_off = pl->pair_off;
    a.pair_m = pl->pair_m;
    a.pair_cls = pl->pair_cls;
    a.ve_off = pl->ve_off;
    a.ve_ids = pl->ve_ids;
    a.f_qp = f_qp;
    a.delta = pl->delta;
    a.psi = pl->psi;
    a.mc_samples = pl->mc;
    a.caps = pl->strategy == NLFEM_FULLCAPS ? 1 : 0;
    a.vr = pl->cap_sampling == NLFEM_CAPS_OUTSIDE_UI ? 1 : 0;
    a.keying = pl->keying;
    a.key0 = (uint32_t)(pl->seed & 0xFFFFFFFFull);
    a.key1 = (uint32_t)(pl->seed >> 32);
    a.fx_shift = pl->fx_shift;
    a.g_shift = pl->g_shift;
    a.w_shift = pl->w_shift;
    a.umax = std::max(pl->umax, 1);
    a.cblk = pl->cblk;
    a.oblk = pl->oblk;
    a.gacc = pl->gacc;
    a.gstride = pl->K;
    a.rglob = pl->rglob;
    a.stab = pl->stab;
    a.stab_stride = pl->stab_stride;
    return a;
}

// numeric phase of one plan after its integration: G_m, then the rows
nlfem_status enqueue_rows(nlfem_ctx* c, nlfem_plan* pl, const double* g_nodal, double* ff_val, double* fc_val,
                          double* rhs, hipStream_t s) {
    HIPCHK(launch_g_finalize(pl->K, pl->region, pl->inner_cnt, pl->vol, pl->gacc, pl->g_shift, pl->w_shift, pl->gvals,
                             s));
    RowPlan rp = make_row_plan(pl);
    RowNumeric nm;
    nm.cblk = pl->cblk;
    nm.oblk = pl->oblk;
    nm.gvals = pl->gvals;
    nm.g_nodal = g_nodal;
    nm.row_shift = pl->row_shift;
    nm.ff_val = ff_val;
    nm.fc_val = fc_val ? fc_val : pl->fc_val_int;
    nm.rhs = rhs;
    if (pl->racc) HIPCHK(launch_row_assemble_global(rp, nm, pl->racc, pl->n_free, s));
    else HIPCHK(launch_row_assemble(rp, nm, pl->n_free, s));
    return NLFEM_OK;
}

// ---------------------------------------------------------------------------
// Autotuner cache: shape class -> (block, workgroups per CU), shared by all
// batches of the process.
struct TuneKey {
    int log2_pairs, log2_items, mc, fp32, per_cu, keying;
    bool operator<(const TuneKey& o) const {
        if (keying != o.keying) return keying < o.keying;
        if (log2_pairs != o.log2_pairs) return log2_pairs < o.log2_pairs;
        if (log2_items != o.log2_items) return log2_items < o.log2_items;
        if (mc != o.mc) return mc < o.mc;
        if (fp32 != o.fp32) return fp32 < o.fp32;
        return per_cu < o.per_cu;
    }
};
struct TuneVal {
    int block, wg_per_cu;  // wg_per_cu 0: one workgroup per item, else a persistent grid of n_cu * wg_per_cu
    double ms;
};
// guarded by tune_mutex(): batches of different threads share the cache
std::mutex& tune_mutex() {
    static std::mutex m;
    return m;
}
std::map<TuneKey, TuneVal>& tune_cache() {
    static std::map<TuneKey, TuneVal> m;
    return m;
}

int ilog2(int64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

}  // namespace

struct nlfem_batch {
    nlfem_ctx* ctx = nullptr;
    std::vector<nlfem_plan*> plans;
    struct Out {
        int64_t* ff_row_ptr;
        int32_t* ff_col;
        double* ff_val;
        int64_t* fc_row_ptr;
        int32_t* fc_col;
        double* fc_val;
        double* rhs;
        int32_t* f2v;
    };
    std::vector<Out> outs;
    std::vector<void*> owned;
    std::vector<IntegrateArgs> descs;
    IntegrateArgs* d_descs = nullptr;
    // Meshes whose local vertex sets allow the same number of resident
    // workgroups per CU (LDS footprint) share one launch, so a mesh with a
    // small horizon is not held to the occupancy of the largest.
    struct Group {
        int umax = 1, per_cu = 1;
        int2* d_items = nullptr;   // (mesh, outer position), longest first
        int2* d_sample = nullptr;  // every stride-th item: the autotuner times this list
        int64_t n_items = 0, n_sample = 0, pairs = 0;
        unsigned long long* d_head = nullptr;  // queue head of the persistent launch
        int block = 256, grid = 0;             // grid 0: one workgroup per item
        double tune_ms = 0.0;
    };
    std::vector<Group> groups;
    int64_t total_pairs = 0;
    int n_cu = 256;
    bool fp32 = false;
    bool vr = false;
    int keying = 0;
    bool tuned = false;
    hipStream_t gs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double*> cap_f, cap_g;
    double last_ms = 0.0;
    std::mutex owned_mu;  // the plan builders allocate outputs concurrently
    void* alloc(size_t b) {
        void* p = dalloc(ctx, b);
        if (p) {
            std::lock_guard<std::mutex> lk(owned_mu);
            owned.push_back(p);
        }
        return p;
    }
};

namespace {

// Per mesh of a batch, with context c (its stream): the output arrays, the
// CSR pattern copied into them, and the pairs per outer tet read back (the
// item costs of the longest-first order) into off.
nlfem_status batch_mesh_out(nlfem_ctx* c, nlfem_batch* b, nlfem_plan* pl, int i, std::vector<int64_t>& off) {
    hipStream_t s = c->stream;
    nlfem_batch::Out& o = b->outs[(size_t)i];
    const int64_t nf = pl->n_free;
    o.ff_row_ptr = (int64_t*)b->alloc((size_t)(nf + 1) * 8);
    o.ff_col = (int32_t*)b->alloc((size_t)(pl->nnz_ff + 1) * 4);
    o.ff_val = (double*)b->alloc((size_t)(pl->nnz_ff + 1) * 8);
    o.fc_row_ptr = (int64_t*)b->alloc((size_t)(nf + 1) * 8);
    o.fc_col = (int32_t*)b->alloc((size_t)(pl->nnz_fc + 1) * 4);
    o.fc_val = (double*)b->alloc((size_t)(pl->nnz_fc + 1) * 8);
    o.rhs = (double*)b->alloc((size_t)(nf + 1) * 8);
    o.f2v = (int32_t*)b->alloc((size_t)(nf + 1) * 4);
    if (!o.ff_row_ptr || !o.ff_col || !o.ff_val || !o.fc_row_ptr || !o.fc_col || !o.fc_val || !o.rhs || !o.f2v)
        return fail(c, NLFEM_E_OOM, owner_err(pl));
    HIPCHK(launch_copy_i64(pl->ff_row_ptr, o.ff_row_ptr, nf + 1, s));
    HIPCHK(launch_copy_i32(pl->ff_col, o.ff_col, pl->nnz_ff, s));
    HIPCHK(launch_copy_i64(pl->fc_row_ptr, o.fc_row_ptr, nf + 1, s));
    HIPCHK(launch_copy_i32(pl->fc_col, o.fc_col, pl->nnz_fc, s));
    HIPCHK(launch_copy_i32(pl->free_to_vertex, o.f2v, nf, s));
    off.resize((size_t)pl->n_outer + 1);
    HIPCHK(hipMemcpyAsync(off.data(), pl->pair_off, off.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return NLFEM_OK;
}

void batch_free(nlfem_batch* b) {
    if (!b) return;
    if (b->gs) hipStreamSynchronize(b->gs);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->ev_in) hipEventDestroy(b->ev_in);
    if (b->ev_out) hipEventDestroy(b->ev_out);
    if (b->gs) hipStreamDestroy(b->gs);
    for (nlfem_plan* p : b->plans) {
        p->release();
        delete p;
    }
    for (void* p : b->owned) dfree(b->ctx, p);
    delete b;
}

// numeric phase of every mesh of the batch on stream s
nlfem_status batch_enqueue(nlfem_batch* b, const double* const* g_nodal, hipStream_t s) {
    nlfem_ctx* c = b->ctx;
    for (nlfem_plan* pl : b->plans) HIPCHK(launch_fill_u64(pl->gacc, 22 * pl->K, s));
    for (const nlfem_batch::Group& g : b->groups) {
        if (g.grid > 0)
            HIPCHK(launch_integrate_batch(b->d_descs, g.d_items, g.n_items, g.d_head, g.umax, b->fp32, b->vr, b->keying, g.block,
                                          g.grid, s));
        else
            HIPCHK(launch_integrate_items(b->d_descs, g.d_items, g.n_items, g.umax, b->fp32, b->vr, b->keying, g.block, s));
    }
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const nlfem_batch::Out& o = b->outs[i];
        nlfem_status st = enqueue_rows(c, b->plans[i], g_nodal ? g_nodal[i] : nullptr, o.ff_val, o.fc_val, o.rhs, s);
        if (st != NLFEM_OK) return st;
    }
    return NLFEM_OK;
}

// integration time of the group's tuning sample with one launch shape
// (grid 0: one workgroup per item)
double time_integrate(nlfem_batch* b, const nlfem_batch::Group& g, int block, int grid) {
    Timer t(b->gs);
    const hipError_t e =
        grid > 0 ? launch_integrate_batch(b->d_descs, g.d_sample, g.n_sample, g.d_head, g.umax, b->fp32, b->vr, b->keying, block,
                                          grid, b->gs)
                 : launch_integrate_items(b->d_descs, g.d_sample, g.n_sample, g.umax, b->fp32, b->vr, b->keying, block, b->gs);
    if (e != hipSuccess) return 1e30;
    return t.stop();
}

}  // namespace

namespace {

// CG on the device (k_cg.hip) with a host poll every kCgPoll iterations: the
// iterations after the stop are no-ops on the device, so *iters is exact.
constexpr int kCgPoll = 8;

nlfem_status cg_solve(nlfem_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                      const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters, double* rel_res,
                      double* work) {
    hipStream_t s = c->stream;
    const CgState* st = cg_state(work, n);
    CgState h;
    auto poll = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(c->pinned, st, kCgPollBytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        std::memcpy(&h, c->pinned, kCgPollBytes);
        return e;
    };
    HIPCHK(cg_enqueue_start(n, row_ptr, col, val, b, x, rtol, max_iter, work, s));
    HIPCHK(poll());
    int queued = 0;
    while (h.done == 0 && queued < max_iter) {
        const int cnt = std::min(kCgPoll, max_iter - queued);
        HIPCHK(cg_enqueue_iterations(n, row_ptr, col, val, x, queued, cnt, work, s));
        queued += cnt;
        HIPCHK(poll());
    }
    if (h.done == 4) {  // b = 0: the solution is 0
        HIPCHK(cg_enqueue_zero(n, x, s));
        HIPCHK(hipStreamSynchronize(s));
        *iters = 0;
        *rel_res = 0.0;
        return NLFEM_OK;
    }
    *iters = h.iter;
    *rel_res = std::sqrt(h.res2) / h.bnorm;
    if (h.done == 2)
        return fail(c, NLFEM_E_NOT_CONVERGED,
                    "CG breakdown after " + std::to_string(h.iter) + " iterations: p.Ap <= 0 or a non-finite value "
                    "(the matrix is not symmetric positive definite)");
    if (h.done != 1) return fail(c, NLFEM_E_NOT_CONVERGED, "CG did not converge");
    return NLFEM_OK;
}

}  // namespace

// ============================================================================
extern "C" {

void nlfem_rule_constants(double* alpha, double* beta) {
    if (alpha) *alpha = kAlpha;
    if (beta) *beta = kBeta;
}

nlfem_status nlfem_create(nlfem_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes) {
    if (!out) return NLFEM_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        hipGetLastError();
        return NLFEM_E_DEVICE;
    }
    if (device < 0 || device >= n) return NLFEM_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return NLFEM_E_DEVICE;
    {
        // the allocation-free CG's device scratch: its address on this device
        void* scratch = nullptr;
        if (cg_noalloc_setup(device, &scratch) != hipSuccess || !scratch) {
            hipGetLastError();
            return NLFEM_E_DEVICE;
        }
    }
    nlfem_ctx* c = new nlfem_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->lds_max = prop.sharedMemPerBlock;
    if (hipHostMalloc((void**)&c->pinned, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->pinned_i, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return NLFEM_E_DEVICE;
    }
    *out = c;
    return NLFEM_OK;
}

nlfem_status nlfem_destroy(nlfem_ctx* c) {
    if (!c) return NLFEM_E_INVALID_ARG;
    hipStreamSynchronize(c->stream);
    if (c->pool) {
        drain_pending(c);
        for (auto& kv : c->sizes) c->pool->release(kv.first, kv.second);
    } else {
        release_cache(c);
        for (auto& kv : c->sizes) hipFree(kv.first);
    }
    c->sizes.clear();
    hipHostFree(c->pinned);
    hipHostFree(c->pinned_i);
    delete c;
    return NLFEM_OK;
}

const char* nlfem_last_error(const nlfem_ctx* c) { return c ? c->err.c_str() : "null context"; }

nlfem_status nlfem_memory_in_use(const nlfem_ctx* c, size_t* bytes) {
    if (!c || !bytes) return NLFEM_E_INVALID_ARG;
    *bytes = c->live + c->cached;
    return NLFEM_OK;
}

nlfem_status nlfem_trim(nlfem_ctx* c) {
    if (!c) return NLFEM_E_INVALID_ARG;
    hipStreamSynchronize(c->stream);
    drain_pending(c);
    release_cache(c);
    return NLFEM_OK;
}

namespace {
nlfem_status plan_create_in(nlfem_ctx* owner, nlfem_ctx* c, const nlfem_mesh* mesh, const nlfem_params* prm,
                            nlfem_plan** out);
}  // namespace

nlfem_status nlfem_plan_create(nlfem_ctx* c, const nlfem_mesh* mesh, const nlfem_params* prm, nlfem_plan** out) {
    if (!c) return NLFEM_E_INVALID_ARG;
    return plan_create_in(c, c, mesh, prm, out);
}

namespace {
// builds the plan with context c (its stream, temporaries and error text);
// the plan's own memory belongs to owner
nlfem_status plan_create_in(nlfem_ctx* owner, nlfem_ctx* c, const nlfem_mesh* mesh, const nlfem_params* prm,
                            nlfem_plan** out) {
    if (!out || !mesh || !prm) return fail(c, NLFEM_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (mesh->n_vertices < 0 || mesh->n_tets < 0) return fail(c, NLFEM_E_INVALID_ARG, "negative mesh size");
    if (mesh->n_tets > 0 && (!mesh->coords || !mesh->tets || !mesh->vertex_free))
        return fail(c, NLFEM_E_INVALID_ARG, "null mesh array");
    if (mesh->mem_kind != 0 && mesh->mem_kind != 1) return fail(c, NLFEM_E_INVALID_ARG, "mem_kind must be 0 or 1");
    if (!(prm->delta > 0.0) || !std::isfinite(prm->delta)) return fail(c, NLFEM_E_INVALID_ARG, "delta must be > 0");
    if (prm->mc_samples < 1 || prm->mc_samples > NLFEM_MAX_MC_SAMPLES)
        return fail(c, NLFEM_E_INVALID_ARG, "mc_samples must be in [1, " + std::to_string(NLFEM_MAX_MC_SAMPLES) + "]");
    if (prm->precision != NLFEM_FP64 && prm->precision != NLFEM_FP32_LOCAL)
        return fail(c, NLFEM_E_INVALID_ARG, "unknown precision");
    if (prm->strategy < NLFEM_FULLCAPS || prm->strategy > NLFEM_BARYCENTER)
        return fail(c, NLFEM_E_INVALID_ARG, "unknown ball approximation strategy");
    if (prm->cap_sampling != NLFEM_CAPS_WHOLE_ELEMENT && prm->cap_sampling != NLFEM_CAPS_OUTSIDE_UI)
        return fail(c, NLFEM_E_INVALID_ARG, "unknown cap sampling mode");
    if (prm->cap_sampling == NLFEM_CAPS_OUTSIDE_UI && prm->mc_samples < 3)
        return fail(c, NLFEM_E_INVALID_ARG, "cap sampling on E_m minus U_I needs mc_samples >= 3");
    if (prm->keying != NLFEM_KEY_PAIR && prm->keying != NLFEM_KEY_ELEMENT)
        return fail(c, NLFEM_E_INVALID_ARG, "unknown Monte Carlo keying");
    if (mesh->n_tets >= (int64_t)1 << 31 || mesh->n_vertices >= (int64_t)1 << 31)
        return fail(c, NLFEM_E_UNSUPPORTED, "mesh larger than 2^31 entities");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "hipSetDevice failed");
    nlfem_plan* pl = new nlfem_plan();
    pl->ctx = owner;
    pl->delta = prm->delta;
    pl->psi = prm->psi;
    pl->mc = prm->mc_samples;
    pl->seed = prm->seed;
    pl->precision = prm->precision;
    pl->strategy = prm->strategy;
    pl->cap_sampling = prm->cap_sampling;
    pl->keying = prm->keying;
    nlfem_status st = build_plan(c, pl, mesh, prm);
    if (st != NLFEM_OK) {
        hipStreamSynchronize(c->stream);
        pl->release();
        delete pl;
        return st;
    }
    *out = pl;
    return NLFEM_OK;
}
}  // namespace

nlfem_status nlfem_plan_info(const nlfem_plan* pl, int64_t* n_free, int64_t* nnz_ff, int64_t* nnz_fc,
                             int64_t pair_counts[5], size_t* workspace_bytes) {
    if (!pl) return NLFEM_E_INVALID_ARG;
    if (n_free) *n_free = pl->n_free;
    if (nnz_ff) *nnz_ff = pl->nnz_ff;
    if (nnz_fc) *nnz_fc = pl->nnz_fc;
    if (pair_counts)
        for (int i = 0; i < 5; ++i) pair_counts[i] = pl->pair_counts[i];
    if (workspace_bytes) {
        size_t b = 0;
        for (void* p : pl->owned) {
            auto it = pl->ctx->sizes.find(p);
            if (it != pl->ctx->sizes.end()) b += it->second;
        }
        *workspace_bytes = b;
    }
    return NLFEM_OK;
}

namespace {

// numeric phase; g_deg < 0: nodal constraint values only
nlfem_status assemble_impl(nlfem_plan* pl, const double* f_qp, const double* g_nodal, int32_t g_deg,
                           const double* g_coef, int64_t* ff_row_ptr, int32_t* ff_col, double* ff_val,
                           int64_t* fc_row_ptr, int32_t* fc_col, double* fc_val, double* rhs,
                           int32_t* free_to_vertex) {
    if (!pl) return NLFEM_E_INVALID_ARG;
    nlfem_ctx* c = pl->ctx;
    if (pl->nnz_ff > 0 && !ff_val) return fail(c, NLFEM_E_INVALID_ARG, "ff_val is required");
    if (pl->n_free > 0 && !rhs) return fail(c, NLFEM_E_INVALID_ARG, "rhs is required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "hipSetDevice failed");
    hipStream_t s = c->stream;
    Timer total(s);
    const int64_t nf = pl->n_free;
    if (ff_row_ptr) HIPCHK(launch_copy_i64(pl->ff_row_ptr, ff_row_ptr, nf + 1, s));
    if (ff_col) HIPCHK(launch_copy_i32(pl->ff_col, ff_col, pl->nnz_ff, s));
    if (fc_row_ptr) HIPCHK(launch_copy_i64(pl->fc_row_ptr, fc_row_ptr, nf + 1, s));
    if (fc_col) HIPCHK(launch_copy_i32(pl->fc_col, fc_col, pl->nnz_fc, s));
    if (free_to_vertex) HIPCHK(launch_copy_i32(pl->free_to_vertex, free_to_vertex, nf, s));
    IntegrateArgs a = make_args(pl, f_qp);
    Timer tint(s);
    HIPCHK(launch_fill_u64(pl->gacc, 22 * pl->K, s));
    HIPCHK(launch_integrate(a, pl->precision == NLFEM_FP32_LOCAL, s));
    if (g_deg >= 0) {
        const size_t nc = (size_t)(g_deg + 1) * (g_deg + 1) * (g_deg + 1);
        TMP(t_coef, nc * sizeof(double));
        // pageable source: the call returns once the host data is staged
        HIPCHK(hipMemcpyAsync(t_coef.p, g_coef, nc * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(launch_exact_g(a, g_nodal, t_coef.as<double>(), g_deg, s));
    }
    pl->times[3] = tint.stop();
    Timer tred(s);
    nlfem_status st = enqueue_rows(c, pl, g_nodal, ff_val, fc_val, rhs, s);
    if (st != NLFEM_OK) return st;
    pl->times[4] = tred.stop();
    pl->times[5] = total.stop();
    return NLFEM_OK;
}

}  // namespace

nlfem_status nlfem_assemble(nlfem_plan* pl, const double* f_qp, const double* g_nodal, int64_t* ff_row_ptr,
                            int32_t* ff_col, double* ff_val, int64_t* fc_row_ptr, int32_t* fc_col, double* fc_val,
                            double* rhs, int32_t* free_to_vertex) {
    return assemble_impl(pl, f_qp, g_nodal, -1, nullptr, ff_row_ptr, ff_col, ff_val, fc_row_ptr, fc_col, fc_val, rhs,
                         free_to_vertex);
}

nlfem_status nlfem_assemble_exact_g(nlfem_plan* pl, const double* f_qp, const double* g_nodal, int32_t g_degree,
                                    const double* g_coef, int64_t* ff_row_ptr, int32_t* ff_col, double* ff_val,
                                    int64_t* fc_row_ptr, int32_t* fc_col, double* fc_val, double* rhs,
                                    int32_t* free_to_vertex) {
    if (!pl) return NLFEM_E_INVALID_ARG;
    nlfem_ctx* c = pl->ctx;
    static_assert(NLFEM_MAX_G_DEGREE == kMaxGDegree, "g degree limit");
    if (g_degree < 0 || g_degree > NLFEM_MAX_G_DEGREE || !g_coef)
        return fail(c, NLFEM_E_INVALID_ARG, "g_degree outside [0, NLFEM_MAX_G_DEGREE] or g_coef null");
    if (pl->cap_sampling != NLFEM_CAPS_WHOLE_ELEMENT)
        return fail(c, NLFEM_E_UNSUPPORTED, "exact g needs whole-element cap sampling");
    return assemble_impl(pl, f_qp, g_nodal, g_degree, g_coef, ff_row_ptr, ff_col, ff_val, fc_row_ptr, fc_col, fc_val,
                         rhs, free_to_vertex);
}

nlfem_status nlfem_plan_timings(const nlfem_plan* pl, double times[6]) {
    if (!pl || !times) return NLFEM_E_INVALID_ARG;
    for (int i = 0; i < 6; ++i) times[i] = pl->times[i];
    return NLFEM_OK;
}

nlfem_status nlfem_debug_pairs(nlfem_plan* pl, int64_t q_begin, int64_t q_end, nlfem_pair_record* out,
                               int64_t out_cap, int64_t* n_written) {
    if (!pl || !n_written) return NLFEM_E_INVALID_ARG;
    nlfem_ctx* c = pl->ctx;
    hipStream_t s = c->stream;
    *n_written = 0;
    if (q_end <= q_begin || pl->n_outer == 0) return NLFEM_OK;
    std::vector<int32_t> oid(pl->n_outer);
    std::vector<int64_t> poff(pl->n_outer + 1);
    HIPCHK(hipMemcpyAsync(oid.data(), pl->outer_ids, oid.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(poff.data(), pl->pair_off, poff.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t nlo = q_begin / 4, nhi = (q_end + 3) / 4;
    int64_t olo = std::lower_bound(oid.begin(), oid.end(), (int32_t)nlo) - oid.begin();
    int64_t ohi = std::lower_bound(oid.begin(), oid.end(), (int32_t)std::min<int64_t>(nhi, INT32_MAX)) - oid.begin();
    if (ohi <= olo) return NLFEM_OK;
    int64_t slots = 4 * (poff[ohi] - poff[olo]);
    TMP(t_S, (size_t)(slots + 1) * 15 * 8);
    TMP(t_qm, (size_t)(slots + 1) * 3 * 4);
    IntegrateArgs a = make_args(pl, nullptr);
    HIPCHK(launch_debug_pairs(a, pl->precision == NLFEM_FP32_LOCAL, olo, ohi, t_S.as<double>(), t_qm.as<int32_t>(), s));
    std::vector<double> S((size_t)slots * 15);
    std::vector<int32_t> qm((size_t)slots * 3);
    HIPCHK(hipMemcpyAsync(S.data(), t_S.p, S.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(qm.data(), t_qm.p, qm.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t cnt = 0;
    for (int64_t i = 0; i < slots; ++i) {
        int32_t q = qm[3 * i], cl = qm[3 * i + 2];
        if (cl == 0 || q < q_begin || q >= q_end) continue;
        if (out && cnt < out_cap) {
            out[cnt].q = q;
            out[cnt].m = qm[3 * i + 1];
            out[cnt].cls = cl;
            out[cnt].pad = 0;
            for (int j = 0; j < 15; ++j) out[cnt].S[j] = S[15 * i + j];
        }
        ++cnt;
    }
    *n_written = cnt;
    if (cnt > out_cap) return fail(c, NLFEM_E_INVALID_ARG, "out_cap too small");
    return NLFEM_OK;
}

nlfem_status nlfem_batch_create(nlfem_ctx* c, int32_t n, const nlfem_mesh* meshes, const nlfem_params* params,
                                nlfem_batch** out) {
    if (!c) return NLFEM_E_INVALID_ARG;
    if (!out || n < 0 || (n > 0 && (!meshes || !params))) return fail(c, NLFEM_E_INVALID_ARG, "bad batch argument");
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i) {
        if (params[i].precision != params[0].precision)
            return fail(c, NLFEM_E_INVALID_ARG, "all meshes of a batch must use the same precision");
        if (params[i].cap_sampling != params[0].cap_sampling)
            return fail(c, NLFEM_E_INVALID_ARG, "all meshes of a batch must use the same cap sampling");
        if (params[i].keying != params[0].keying)
            return fail(c, NLFEM_E_INVALID_ARG, "all meshes of a batch must use the same Monte Carlo keying");
    }
    nlfem_batch* b = new nlfem_batch();
    b->ctx = c;
    // frees the partial batch on every early return (including HIPCHK's)
    struct Guard {
        nlfem_batch* b;
        ~Guard() {
            if (b) batch_free(b);
        }
    } guard{b};
    b->fp32 = n > 0 && params[0].precision == NLFEM_FP32_LOCAL;
    b->vr = n > 0 && params[0].cap_sampling == NLFEM_CAPS_OUTSIDE_UI;
    b->keying = n > 0 ? params[0].keying : 0;
    hipDeviceProp_t prop;
    size_t lds_cu = 160 * 1024;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        b->n_cu = prop.multiProcessorCount;
        if (prop.maxSharedMemoryPerMultiProcessor > 0) lds_cu = prop.maxSharedMemoryPerMultiProcessor;
    }
    std::vector<std::vector<int64_t>> offs;  // per mesh: its pair_off on the host
    {
        // The symbolic phases of the meshes are independent: kBuilders threads
        // build them, each with a context of its own (stream, temporaries),
        // taking meshes in turn; the plans' memory belongs to c.  c's cached
        // blocks must be idle before other streams may take them.
        const int nb = n >= 8 ? kBuilders : 1;
        std::vector<nlfem_plan*> plans((size_t)n, nullptr);
        b->outs.resize((size_t)n);
        offs.resize((size_t)n);
        if (nb == 1) {
            for (int32_t i = 0; i < n; ++i) {
                nlfem_status st = nlfem_plan_create(c, &meshes[i], &params[i], &plans[(size_t)i]);
                if (st == NLFEM_OK) st = batch_mesh_out(c, b, plans[(size_t)i], i, offs[(size_t)i]);
                if (st != NLFEM_OK) {
                    for (nlfem_plan* pl : plans) nlfem_plan_destroy(pl);
                    return st;
                }
            }
        } else {
            if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "stream sync failed");
            std::atomic<int> next{0};
            std::atomic<bool> failed{false};
            std::mutex emu;
            nlfem_status first = NLFEM_OK;
            std::string first_msg;
            // each builder's context and stream, kept until all have ended
            std::vector<nlfem_ctx*> wctx((size_t)nb, nullptr);
            std::vector<hipStream_t> wstream((size_t)nb, nullptr);
            auto worker = [&](int w) {
                nlfem_status st = NLFEM_OK;
                std::string msg;
                hipStream_t& ws = wstream[(size_t)w];
                nlfem_ctx*& wc = wctx[(size_t)w];
                if (hipSetDevice(c->device) != hipSuccess ||
                    hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) {
                    (void)hipGetLastError();
                    st = NLFEM_E_DEVICE;
                    msg = "could not create a stream for a plan builder";
                } else if ((st = nlfem_create(&wc, c->device, ws, c->budget)) != NLFEM_OK) {
                    msg = "could not create a plan builder context";
                }
                while (st == NLFEM_OK && !failed.load()) {
                    const int i = next.fetch_add(1);
                    if (i >= n) break;
                    st = plan_create_in(c, wc, &meshes[i], &params[i], &plans[(size_t)i]);
                    if (st == NLFEM_OK) st = batch_mesh_out(wc, b, plans[(size_t)i], i, offs[(size_t)i]);
                    if (st != NLFEM_OK) msg = wc->err;
                }
                // its temporaries are idle once its stream has drained
                if (ws) (void)hipStreamSynchronize(ws);
                if (st != NLFEM_OK) {
                    failed.store(true);
                    std::lock_guard<std::mutex> lk(emu);
                    if (first == NLFEM_OK) {
                        first = st;
                        first_msg = msg;
                    }
                }
            };
            std::vector<std::thread> th;
            for (int w = 0; w < nb; ++w) th.emplace_back(worker, w);
            for (auto& t : th) t.join();
            // after a build that succeeded, the batch's context keeps the
            // builders' cached temporaries (freeing them while the builders
            // ran would have made each wait for the whole device); after a
            // failure they go back to the device with the builders' contexts
            for (int w = 0; w < nb; ++w) {
                nlfem_ctx* wc = wctx[(size_t)w];
                if (wc) {
                    if (first == NLFEM_OK && !c->pool) adopt_cache(c, wc);
                    nlfem_destroy(wc);
                }
                if (wstream[(size_t)w]) (void)hipStreamDestroy(wstream[(size_t)w]);
            }
            if (first != NLFEM_OK) {
                for (nlfem_plan* pl : plans) nlfem_plan_destroy(pl);
                return fail(c, first, first_msg);
            }
        }
        b->plans = plans;
    }
    hipStream_t s = c->stream;
    // resident 256-thread workgroups per CU that the LDS footprint allows,
    // capped at the 3 the register budget allows
    auto per_cu = [&](int umax) {
        const size_t bytes = integrate_lds_bytes(std::max(umax, 1));
        return (int)std::max<size_t>(1, std::min<size_t>(3, lds_cu / bytes));
    };
    std::map<int, int> gid;  // per_cu -> group
    for (int32_t i = 0; i < n; ++i) gid[per_cu(b->plans[i]->umax)] = 0;
    for (auto& kv : gid) {
        kv.second = (int)b->groups.size();
        b->groups.emplace_back();
        b->groups.back().per_cu = kv.first;
    }
    std::vector<std::vector<int2>> items(b->groups.size());
    std::vector<std::vector<int64_t>> cost(b->groups.size());
    for (int32_t i = 0; i < n; ++i) {
        nlfem_plan* pl = b->plans[i];
        b->descs.push_back(make_args(pl, nullptr));
        const int g = gid[per_cu(pl->umax)];
        b->groups[g].umax = std::max(b->groups[g].umax, std::max(pl->umax, 1));
        b->groups[g].pairs += pl->P;
        const std::vector<int64_t>& off = offs[(size_t)i];
        for (int64_t oi = 0; oi < pl->n_outer; ++oi) {
            items[g].push_back(make_int2(i, (int)oi));
            cost[g].push_back(off[oi + 1] - off[oi]);
        }
        b->total_pairs += pl->P;
    }
    // the kernel lays out LDS from the descriptor's umax: every mesh of a
    // group uses the group's
    for (int32_t i = 0; i < n; ++i) b->descs[i].umax = b->groups[gid[per_cu(b->plans[i]->umax)]].umax;
    for (size_t g = 0; g < b->groups.size(); ++g) {
        nlfem_batch::Group& G = b->groups[g];
        if (integrate_lds_bytes(G.umax) > c->lds_max) {
            return fail(c, NLFEM_E_UNSUPPORTED, "batch ball vertex set too large for LDS");
        }
        // longest items first
        std::vector<int64_t> order(items[g].size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t bb) { return cost[g][a] > cost[g][bb]; });
        std::vector<int2> sorted(items[g].size());
        for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[g][order[i]];
        G.n_items = (int64_t)sorted.size();
        if (G.n_items > 0x7fffffff) {
            return fail(c, NLFEM_E_UNSUPPORTED, "more than 2^31-1 outer tets in one batch group");
        }
        // tuning sample: a strided subset of the longest-first list with about
        // 1.5e8 pairs, so each candidate shape is timed on the same mix of
        // item costs in a fraction of the full launch
        const int64_t stride = std::min<int64_t>(64, std::max<int64_t>(1, G.pairs / 150000000));
        std::vector<int2> sample;
        for (size_t i = 0; i < sorted.size(); i += (size_t)stride) sample.push_back(sorted[i]);
        G.n_sample = (int64_t)sample.size();
        G.d_sample = (int2*)b->alloc(sample.size() * sizeof(int2) + 16);
        G.d_items = (int2*)b->alloc(sorted.size() * sizeof(int2) + 16);
        G.d_head = (unsigned long long*)b->alloc(64);
        if (!G.d_items || !G.d_sample || !G.d_head) {
            return fail(c, NLFEM_E_OOM, c->err);
        }
        if (!sorted.empty()) {
            HIPCHK(hipMemcpyAsync(G.d_items, sorted.data(), sorted.size() * sizeof(int2), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(G.d_sample, sample.data(), sample.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        }
        // the host vectors are freed at the end of this scope: finish the copies first
        HIPCHK(hipStreamSynchronize(s));
    }
    b->d_descs = (IntegrateArgs*)b->alloc(b->descs.size() * sizeof(IntegrateArgs) + 16);
    if (!b->d_descs) {
        return fail(c, NLFEM_E_OOM, c->err);
    }
    if (!b->descs.empty())
        HIPCHK(hipMemcpyAsync(b->d_descs, b->descs.data(), b->descs.size() * sizeof(IntegrateArgs),
                              hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        return fail(c, NLFEM_E_DEVICE, "stream/event creation failed");
    }
    guard.b = nullptr;
    *out = b;
    return NLFEM_OK;
}

nlfem_status nlfem_batch_info(const nlfem_batch* b, int32_t i, int64_t* n_free, int64_t* nnz_ff, int64_t* nnz_fc,
                              int64_t pair_counts[5]) {
    if (!b || i < 0 || i >= (int32_t)b->plans.size()) return NLFEM_E_INVALID_ARG;
    return nlfem_plan_info(b->plans[i], n_free, nnz_ff, nnz_fc, pair_counts, nullptr);
}

nlfem_status nlfem_batch_assemble(nlfem_batch* b, const double* const* f_qp, const double* const* g_nodal) {
    if (!b) return NLFEM_E_INVALID_ARG;
    nlfem_ctx* c = b->ctx;
    const size_t n = b->plans.size();
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "hipSetDevice failed");
    // inputs: f pointers live in the device descriptors (updated outside the graph)
    bool fchanged = false;
    for (size_t i = 0; i < n; ++i) {
        const double* f = f_qp ? f_qp[i] : nullptr;
        if (b->descs[i].f_qp != f) {
            b->descs[i].f_qp = f;
            fchanged = true;
        }
    }
    HIPCHK(hipEventRecord(b->ev_in, c->stream));
    HIPCHK(hipStreamWaitEvent(b->gs, b->ev_in, 0));
    if (fchanged && n)
        HIPCHK(hipMemcpyAsync(b->d_descs, b->descs.data(), n * sizeof(IntegrateArgs), hipMemcpyHostToDevice, b->gs));
    if (!b->tuned) {
        for (nlfem_batch::Group& G : b->groups) {
            TuneKey key{ilog2(std::max<int64_t>(G.pairs, 1)), ilog2(std::max<int64_t>(G.n_items, 1)),
                        n ? b->plans[0]->mc : 0, b->fp32 ? 1 : 0, G.per_cu, b->keying};
            TuneVal tv{0, 0, 0.0};
            {
                std::lock_guard<std::mutex> lk(tune_mutex());
                auto it = tune_cache().find(key);
                if (it != tune_cache().end()) tv = it->second;
            }
            if (tv.block == 0) {
                // timed outside the lock; a concurrent batch of the same class
                // may time it too, and either result is a valid choice.
                // Candidates: a persistent grid of 2, 3, 4 or 6 workgroups per
                // CU (at most 12 waves per CU), or one workgroup per item.
                tv = TuneVal{256, 0, 1e30};
                const int blocks[2] = {128, 256};
                const int wpc[5] = {2, 3, 4, 6, 0};
                for (int bi = 0; bi < 2; ++bi)
                    for (int wi = 0; wi < 5; ++wi) {
                        if ((blocks[bi] / 64) * wpc[wi] > 12) continue;
                        const double ms = time_integrate(b, G, blocks[bi], b->n_cu * wpc[wi]);
                        if (ms < tv.ms) tv = TuneVal{blocks[bi], wpc[wi], ms};
                    }
                std::lock_guard<std::mutex> lk(tune_mutex());
                tune_cache().emplace(key, tv);
            }
            G.block = tv.block;
            G.grid = b->n_cu * tv.wg_per_cu;
            G.tune_ms = tv.ms;
        }
        b->tuned = true;
    }
    std::vector<const double*> gcur(n);
    for (size_t i = 0; i < n; ++i) gcur[i] = g_nodal ? g_nodal[i] : nullptr;
    if (!b->exec || gcur != b->cap_g) {
        if (b->exec) {
            hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
        nlfem_status st = batch_enqueue(b, gcur.data(), b->gs);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(b->gs, &g);
        if (st != NLFEM_OK) return st;
        if (ee != hipSuccess) return fail(c, NLFEM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
        b->graph = g;
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->cap_g = gcur;
    }
    Timer t(b->gs);
    HIPCHK(hipGraphLaunch(b->exec, b->gs));
    b->last_ms = t.stop();
    HIPCHK(hipEventRecord(b->ev_out, b->gs));
    HIPCHK(hipStreamWaitEvent(c->stream, b->ev_out, 0));
    return NLFEM_OK;
}

nlfem_status nlfem_batch_system(const nlfem_batch* b, int32_t i, const int64_t** ff_row_ptr, const int32_t** ff_col,
                                const double** ff_val, const int64_t** fc_row_ptr, const int32_t** fc_col,
                                const double** fc_val, const double** rhs, const int32_t** free_to_vertex) {
    if (!b || i < 0 || i >= (int32_t)b->plans.size()) return NLFEM_E_INVALID_ARG;
    const nlfem_batch::Out& o = b->outs[i];
    if (ff_row_ptr) *ff_row_ptr = o.ff_row_ptr;
    if (ff_col) *ff_col = o.ff_col;
    if (ff_val) *ff_val = o.ff_val;
    if (fc_row_ptr) *fc_row_ptr = o.fc_row_ptr;
    if (fc_col) *fc_col = o.fc_col;
    if (fc_val) *fc_val = o.fc_val;
    if (rhs) *rhs = o.rhs;
    if (free_to_vertex) *free_to_vertex = o.f2v;
    return NLFEM_OK;
}

nlfem_status nlfem_batch_tuning(const nlfem_batch* b, int32_t* block, int32_t* grid, double* tuned_integrate_ms,
                                double* last_graph_ms) {
    if (!b) return NLFEM_E_INVALID_ARG;
    // workgroup size of the group with the most pairs and its number of
    // workgroups (the persistent grid, or one per work item); time summed
    // over the groups
    const nlfem_batch::Group* top = nullptr;
    double ms = 0.0;
    for (const nlfem_batch::Group& G : b->groups) {
        ms += G.tune_ms;
        if (!top || G.pairs > top->pairs) top = &G;
    }
    if (block) *block = top ? top->block : 0;
    if (grid) *grid = top ? (top->grid > 0 ? top->grid : (int32_t)std::min<int64_t>(top->n_items, 0x7fffffff)) : 0;
    if (tuned_integrate_ms) *tuned_integrate_ms = ms;
    if (last_graph_ms) *last_graph_ms = b->last_ms;
    return NLFEM_OK;
}

nlfem_status nlfem_batch_set_launch(nlfem_batch* b, int32_t block, int32_t wg_per_cu) {
    if (!b) return NLFEM_E_INVALID_ARG;
    nlfem_ctx* c = b->ctx;
    if (block != 128 && block != 256) return fail(c, NLFEM_E_INVALID_ARG, "block must be 128 or 256");
    if (wg_per_cu < 0 || (block / 64) * wg_per_cu > 12)
        return fail(c, NLFEM_E_INVALID_ARG, "wg_per_cu outside [0, 12 / waves per workgroup]");
    // the next nlfem_batch_assemble uses this shape for every group and
    // captures its graph again
    if (b->gs) HIPCHK(hipStreamSynchronize(b->gs));
    for (nlfem_batch::Group& G : b->groups) {
        G.block = block;
        G.grid = b->n_cu * wg_per_cu;
        G.tune_ms = 0.0;
    }
    b->tuned = true;
    if (b->exec) {
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    return NLFEM_OK;
}

nlfem_status nlfem_batch_destroy(nlfem_batch* b) {
    if (!b) return NLFEM_E_INVALID_ARG;
    batch_free(b);
    return NLFEM_OK;
}

nlfem_status nlfem_plan_destroy(nlfem_plan* pl) {
    if (!pl) return NLFEM_E_INVALID_ARG;
    hipStreamSynchronize(pl->ctx->stream);
    pl->release();
    delete pl;
    return NLFEM_OK;
}

nlfem_status nlfem_cg(nlfem_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                      const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters, double* rel_res) {
    if (!c) return NLFEM_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!row_ptr || !col || !val || !b || !x)) || !iters || !rel_res)
        return fail(c, NLFEM_E_INVALID_ARG, "bad CG argument");
    *iters = 0;
    *rel_res = 0.0;
    if (n == 0) return NLFEM_OK;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "hipSetDevice failed");
    TMP(t_v, cg_work_doubles(n) * sizeof(double));
    return cg_solve(c, n, row_ptr, col, val, b, x, rtol, max_iter, iters, rel_res, t_v.as<double>());
}

nlfem_status nlfem_cg_noalloc(nlfem_ctx* c, int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                              const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters,
                              double* rel_res) {
    if (!c) return NLFEM_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!row_ptr || !col || !val || !b || !x)) || !iters || !rel_res)
        return fail(c, NLFEM_E_INVALID_ARG, "bad CG argument");
    if (n > kCgNoAllocMaxN)
        return fail(c, NLFEM_E_UNSUPPORTED, "nlfem_cg_noalloc: n = " + std::to_string(n) + " exceeds its maximum " +
                                                std::to_string(kCgNoAllocMaxN) + " (use nlfem_cg)");
    *iters = 0;
    *rel_res = 0.0;
    if (n == 0) return NLFEM_OK;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLFEM_E_DEVICE, "hipSetDevice failed");
    double* work = (double*)cg_noalloc_scratch(c->device);
    if (!work) return fail(c, NLFEM_E_DEVICE, "nlfem_cg_noalloc: device scratch not resolved for this device");
    return cg_solve(c, n, row_ptr, col, val, b, x, rtol, max_iter, iters, rel_res, work);
}

nlfem_status nlfem_plan_cg(nlfem_plan* pl, const double* ff_val, const double* rhs, double* x, double rtol,
                           int32_t max_iter, int32_t* iters, double* rel_res) {
    if (!pl) return NLFEM_E_INVALID_ARG;
    return nlfem_cg(pl->ctx, pl->n_free, pl->ff_row_ptr, pl->ff_col, ff_val, rhs, x, rtol, max_iter, iters, rel_res);
}

}  // extern "C"
