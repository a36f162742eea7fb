/*
 * nlfem.h -- C ABI of the MI355X (gfx950) library that assembles the 3D P1
 * finite-element system of the volume-constrained nonlocal Poisson problem
 * with a constant kernel on the horizon ball, using the "fullcaps" ball
 * approximation, and solves it by conjugate gradients.
 *
 * Paper: G. Chen, Y. Ma, J. Zhang, "High performance implementation of 3D FEM
 * for nonlocal Poisson problem with different ball approximation strategies".
 *
 * Conventions for every entry point:
 *   - All functions return nlfem_status; nothing throws across the ABI.
 *   - After a failure, nlfem_last_error(ctx) holds a message (owned by the
 *     context, valid until the next call on that context).
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary CPU memory.  Which one a pointer is, is
 *     stated per argument (mesh arrays: by nlfem_mesh.mem_kind).
 *   - The library never frees caller memory.  Plans own their internal
 *     device buffers and free them in nlfem_plan_destroy.
 *   - Work is issued on the context's stream; entry points that return sizes
 *     or scalars to the host synchronise that stream.
 */
#ifndef NLFEM_H
#define NLFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nlfem_ctx nlfem_ctx;
typedef struct nlfem_plan nlfem_plan;

/* Largest N: the sample sums are exact integers (count and sum L_j in 32 bits,
 * sum L_i L_j in 64 bits), which needs N * 2^21 < 2^32.                       */
#define NLFEM_MAX_MC_SAMPLES 2047

/* Largest per-axis degree of the polynomial g of nlfem_assemble_exact_g.   */
#define NLFEM_MAX_G_DEGREE 4

typedef enum {
    NLFEM_OK = 0,
    NLFEM_E_INVALID_ARG = 1,   /* null pointer, delta <= 0, N outside [1, 2047], unknown strategy or
                                  cap sampling, negative size                                    */
    NLFEM_E_MESH = 2,          /* index out of range, zero-volume tet, free vertex in a T_OmegaI tet */
    NLFEM_E_OOM = 3,           /* allocation failed or would exceed the context's HBM budget  */
    NLFEM_E_DEVICE = 4,        /* a HIP runtime call failed                                  */
    NLFEM_E_NOT_CONVERGED = 5, /* CG hit max_iter; x and the residual are still written     */
    NLFEM_E_UNSUPPORTED = 6    /* a size beyond what this build handles (message says which) */
} nlfem_status;

typedef enum {
    NLFEM_FP64 = 0,       /* every step in IEEE double                                        */
    NLFEM_FP32_LOCAL = 1  /* per-pair subtet rule in float; classification, sample acceptance,
                             the (exact, integer) sample sums and all global sums as in FP64.
                             No faster than NLFEM_FP64 on gfx950: without packed FP32, a float
                             FMA issues like a double one, and the sample test that dominates
                             must decide acceptance as the FP64 form does; kept as the
                             stated-accuracy form (about 1e-7 of the row scale)            */
} nlfem_precision;

/* Ball approximation strategy (Sec. 4.1: which elements, or element pieces,
 * make up the approximate ball B_delta,h(x) of an outer point x).           */
typedef enum {
    NLFEM_FULLCAPS = 0,   /* inside elements whole, T_I of the cut ones (subdivision of conv(I u P)),
                             and the fullcaps (E - U_I) n B by Monte Carlo (Sec. 4.2.2); default  */
    NLFEM_NOCAPS = 1,     /* inside elements and T_I only (Def. nocaps); no Monte Carlo          */
    NLFEM_OVERLAP = 2,    /* every element that meets the ball, whole                           */
    NLFEM_INSIDE = 3,     /* only the elements with all vertices inside the ball, whole          */
    NLFEM_BARYCENTER = 4  /* the elements whose barycenter ((X0+X1)+(X2+X3))/4 lies in the ball  */
} nlfem_strategy;

/* Where the fullcaps Monte Carlo samples are drawn (strategy fullcaps only).  */
typedef enum {
    NLFEM_CAPS_WHOLE_ELEMENT = 0, /* uniform on E_m, rejecting U_I (default)                        */
    NLFEM_CAPS_OUTSIDE_UI = 1     /* uniform on E_m minus U_I, no U_I test: for n_in = 3 the corner
                                     tet at the outside vertex; for n_in = 1, 2 the three cone tets
                                     from the first outside vertex over the region's far faces,
                                     tet j taking the samples floor(j N/3) <= s < floor((j+1) N/3)
                                     at weight |T_j| / N_j; CUT(0) as the default.  Same
                                     expectation, lower variance (Sec. 4.2.2 leaves the sampling
                                     open); needs mc_samples >= 3 (else NLFEM_E_INVALID_ARG)      */
} nlfem_cap_sampling;

/* Which Philox counters key the fullcaps Monte Carlo samples (Sec. 4.2.2
 * leaves the sampling method open).  Sample pair j = floor(s / 2) of the pair
 * (outer point q = 4 n + k, element m) uses counter
 *   NLFEM_KEY_PAIR:    (q, m, j, 0) -- N samples of its own for every pair;
 *   NLFEM_KEY_ELEMENT: (m, j, 0, 1) -- N samples per element, the same points
 *                      of E_m for every outer point (correlated across
 *                      points, unbiased for each).  With the whole-element
 *                      cap sampling the plan draws them once into a table
 *                      of 8 bytes per sample and element (K x round8(N + 8)
 *                      words of device memory held by the plan) that the
 *                      integration reads instead of drawing per pair.        */
typedef enum {
    NLFEM_KEY_PAIR = 0,
    NLFEM_KEY_ELEMENT = 1
} nlfem_keying;

/* Tetrahedral mesh of Omega u Omega_I (Sec. 3.1: coinciding triangulations of
 * Omega and Omega_I; P1 nodes on the boundary of Omega and in Omega_I carry the
 * volume constraint, Sec. 3.2).                                              */
typedef struct {
    int64_t n_vertices, n_tets;
    const double *coords;        /* [n_vertices][3] vertex coordinates                               */
    const int32_t *tets;         /* [n_tets][4] 0-based vertex ids, either orientation                */
    const uint8_t *vertex_free;  /* [n_vertices] 1 = unknown (node in open Omega), 0 = constrained    */
    const uint8_t *tet_region;   /* optional [n_tets]: 1 = T_Omega, 0 = T_OmegaI; NULL = T_Omega iff
                                    the tet has a free vertex                                        */
    int32_t mem_kind;            /* 0: the arrays above are host memory; 1: device memory             */
} nlfem_mesh;

/* Method parameters (Sec. 2.1 kernel gamma = psi * indicator of B_delta(x);
 * Sec. 4.2.2 fullcaps with N Monte Carlo samples per cut (point, element) pair,
 * or per cut element with element keying). */
typedef struct {
    double delta;                /* horizon > 0                                                       */
    double psi;                  /* kernel constant; the operator is L u = 2 int_B (u(y)-u(x)) psi dy */
    int32_t mc_samples;          /* N uniform samples per cut pair, 1 <= N <= NLFEM_MAX_MC_SAMPLES  */
    uint64_t seed;               /* Philox4x32-10 key                                                 */
    int32_t precision;           /* nlfem_precision                                                   */
    const uint8_t *outer_mask;   /* optional [n_tets], same memory kind as the mesh: 1 = use this tet
                                    as an outer element (subset runs); NULL = all T_Omega tets        */
    int32_t strategy;            /* nlfem_strategy (0 = fullcaps)                                     */
    int32_t cap_sampling;        /* nlfem_cap_sampling (0 = whole element)                            */
    int32_t keying;              /* nlfem_keying (0 = per pair); unknown values: NLFEM_E_INVALID_ARG  */
} nlfem_params;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  hbm_budget_bytes caps the device
 * memory the library may hold at once (0 = no cap).                          */
nlfem_status nlfem_create(nlfem_ctx **ctx, int device, void *hip_stream, size_t hbm_budget_bytes);
/* Frees the context and every device buffer it holds.  Destroy the context's
 * plans first: a plan must not be used or destroyed after its context.      */
nlfem_status nlfem_destroy(nlfem_ctx *ctx);
const char *nlfem_last_error(const nlfem_ctx *ctx);
/* Device memory currently held by the context (plans and cached scratch).   */
nlfem_status nlfem_memory_in_use(const nlfem_ctx *ctx, size_t *bytes);
/* Releases cached scratch blocks the context keeps for reuse.               */
nlfem_status nlfem_trim(nlfem_ctx *ctx);

/* The library's own copies of the 4-point rule constants alpha, beta
 * (Sec. 4.2.1: degree-2, 4 points, equal weights), for checks.                */
void nlfem_rule_constants(double *alpha, double *beta);

/* ---- symbolic phase ------------------------------------------------------ */

/* Validates the mesh, builds the device mesh layout and a uniform-grid cell
 * list, classifies every (outer quadrature point, tet) pair against the open
 * ball exactly in FP64 (IN / CUT(n_in) / OUT; Def. "simplex's dividing
 * strategy"), and builds the local vertex set of every outer tet, the
 * vertex-keyed lists that gather each matrix row, and the CSR pattern of the
 * free rows.  Mesh and mask are read during the call only.  The call's
 * temporaries (the largest: the CSR pattern's row buffer, at least
 * 8 |Ve|max bytes per free row, |Ve|max the largest local vertex set) go back
 * to the context's cache when it returns; nlfem_trim releases them.
 * Horizons whose local vertex sets or matrix rows do not fit in LDS (in 3D
 * about delta > 5h) keep those fixed-point sums in device memory instead
 * (slower, the same results); the environment variable NLFEM_GLOBAL_SUMS=1
 * forces that form for any plan (for checks).  Batches need the LDS form.
 * NLFEM_ROW_STRIDE=<words> (a power of two, for checks) starts the CSR
 * pattern's row buffer that narrow, so that its overflow retry runs, and
 * NLFEM_VE_STRIDE=<entries> sets the local vertex sets' hand-off buffer, so
 * that sets longer than it take the fill pass.                               */
nlfem_status nlfem_plan_create(nlfem_ctx *ctx, const nlfem_mesh *mesh, const nlfem_params *params,
                               nlfem_plan **plan);

/* Sizes for the caller's output buffers (host scalars).
 * pair_counts[5] = number of (point, element) pairs that are IN, CUT(0),
 * CUT(1), CUT(2), CUT(3).  workspace_bytes = device memory held by the plan. */
nlfem_status nlfem_plan_info(const nlfem_plan *plan, int64_t *n_free, int64_t *nnz_ff,
                             int64_t *nnz_fc, int64_t pair_counts[5], size_t *workspace_bytes);

/* ---- numeric phase ------------------------------------------------------- */

/* Assembles A_ff (free x free, free-renumbered), A_fc (free rows x constrained
 * columns, original vertex ids) and b = F_h - A_fc g  (eq. modified_linear:
 * A_h of eq. Ah over the fullcaps ball, F_h of eq. Fh with the nodal volume
 * constraint).  Free vertices are numbered in increasing vertex id; rows and
 * columns are sorted ascending.  All arrays are DEVICE memory owned by the
 * caller and sized from nlfem_plan_info:
 *   f_qp [n_tets][4] f at the 4 outer points of each tet (NULL = 0)
 *   g_nodal [n_vertices] constraint values (only constrained ones read; NULL = 0)
 *   ff_row_ptr [n_free+1], ff_col [nnz_ff], ff_val [nnz_ff]
 *   fc_row_ptr [n_free+1], fc_col [nnz_fc], fc_val [nnz_fc]   (all three NULL to skip)
 *   rhs [n_free], free_to_vertex [n_free] (NULL to skip).
 * Deterministic: the same inputs give bitwise the same outputs.             */
nlfem_status nlfem_assemble(nlfem_plan *plan, const double *f_qp, const double *g_nodal,
                            int64_t *ff_row_ptr, int32_t *ff_col, double *ff_val,
                            int64_t *fc_row_ptr, int32_t *fc_col, double *fc_val, double *rhs,
                            int32_t *free_to_vertex);

/* As nlfem_assemble, with the paper-exact right-hand side: the inner integral
 * of g over Omega_I n B_{delta,h}(x) in F_h (eq. Fh) uses g itself at the
 * inner integration points (the 4-point rule of Sec. 4.2.1 on each IN
 * element and T_I subtet, and the accepted Monte Carlo samples of the caps)
 * instead of its nodal interpolant, and b = F_h - sum over the constraint
 * nodes on the boundary of Omega of A_h(phi_j, phi_i) g_j (eq. F1.5).  The
 * matrix blocks are those of nlfem_assemble (A_fc keeps its nodal form); b
 * differs from nlfem_assemble's by 2 psi sum w phi_i(p) int (g - g_h).
 * g is the tensor polynomial, a HOST array read during the call:
 *   g(y) = sum_{a,b,c = 0..g_degree} g_coef[a + n1 (b + n1 c)] y1^a y2^b y3^c,
 *   n1 = g_degree + 1, 0 <= g_degree <= NLFEM_MAX_G_DEGREE;
 * g_nodal must hold g at the constrained vertices.  Plans with cap sampling
 * NLFEM_CAPS_OUTSIDE_UI are rejected (NLFEM_E_UNSUPPORTED).                  */
nlfem_status nlfem_assemble_exact_g(nlfem_plan *plan, const double *f_qp, const double *g_nodal,
                                    int32_t g_degree, const double *g_coef,
                                    int64_t *ff_row_ptr, int32_t *ff_col, double *ff_val,
                                    int64_t *fc_row_ptr, int32_t *fc_col, double *fc_val, double *rhs,
                                    int32_t *free_to_vertex);

/* Unpreconditioned FP64 conjugate gradients on a CSR matrix (DEVICE arrays):
 * the solve of the free-node system that ends the main assembly algorithm
 * (Sec. 4.3).  x holds x0 on entry and the solution on exit.  Stops when
 * ||r||_2 <= rtol ||b||_2 or after max_iter iterations (host scalars out:
 * *iters = iterations done, *rel_residual = ||r||_2 / ||b||_2 of the last
 * recursively updated residual).  The step lengths, norms and the stopping
 * decision stay on the device; the host polls them every 8 iterations and
 * the iteration count is exact.  b = 0 gives x = 0.  Returns
 * NLFEM_E_NOT_CONVERGED (x and the residual still written) at the cap, and
 * also on a breakdown, p.Ap <= 0 or a non-finite value (the matrix is not
 * symmetric positive definite); the message says which.  Work vectors (3 n
 * doubles) are allocated from the context.                                   */
nlfem_status nlfem_cg(nlfem_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                      const double *val, const double *b, double *x, double rtol, int32_t max_iter,
                      int32_t *iters, double *rel_residual);

/* nlfem_cg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, bitwise the same results, but its work vectors live in a
 * static device array of the library (one per GPU, about 12.6 MB, held until
 * the process ends) instead of context allocations; it calls no hipMalloc or
 * hipFree.  n must be at most 524288 (2^19), else NLFEM_E_UNSUPPORTED.  All
 * calls on one GPU share that array: calls that overlap on one GPU (from
 * several threads or streams) race and must be serialised by the caller.
 * Each call initialises the state it reads, so nothing carries over.         */
nlfem_status nlfem_cg_noalloc(nlfem_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                              const double *val, const double *b, double *x, double rtol, int32_t max_iter,
                              int32_t *iters, double *rel_residual);

/* nlfem_cg on the plan's own A_ff pattern (row pointers and columns as
 * nlfem_assemble writes them, n = n_free) with the caller's DEVICE values
 * ff_val [nnz_ff], right-hand side rhs [n_free] and x [n_free].              */
nlfem_status nlfem_plan_cg(nlfem_plan *plan, const double *ff_val, const double *rhs, double *x, double rtol,
                           int32_t max_iter, int32_t *iters, double *rel_residual);

nlfem_status nlfem_plan_destroy(nlfem_plan *plan);

/* ---- introspection for tests ---------------------------------------------
 * Per-pair records for the outer points q in [q_begin, q_end) where q = 4 n + k
 * indexes the k-th outer point of mesh tet n.  Each record (HOST memory) is
 * nlfem_pair_record; pairs with class OUT are not listed.  *n_written gets the
 * number of records; if out_cap is too small, NLFEM_E_INVALID_ARG is returned
 * and *n_written holds the count needed.                                    */
typedef struct {
    int32_t q;            /* outer point id 4 n + k                                        */
    int32_t m;            /* inner tet id                                                  */
    int32_t cls;          /* 1 IN, 2 + n_in CUT(n_in)                                      */
    int32_t pad;
    double S[15];         /* moments of lambda^m over E_m n B_{delta,h}(p_q):
                             S0, S1[0..3], S2 upper triangle 00,01,02,03,11,12,13,22,23,33 */
} nlfem_pair_record;

nlfem_status nlfem_debug_pairs(nlfem_plan *plan, int64_t q_begin, int64_t q_end,
                               nlfem_pair_record *out, int64_t out_cap, int64_t *n_written);

/* ---- batching ----------------------------------------------------------------
 * Many independent meshes of uneven size and horizon assembled together
 * (the parallel assembly of Sec. 4.4 extended across problems).  The
 * symbolic phase runs per mesh as in nlfem_plan_create.  The numeric phase
 * groups the meshes by how many integration workgroups fit on a CU next to
 * their local vertex set in LDS (1, 2 or 3); each group is ONE integration
 * launch over its (mesh, outer tet) work items, longest first: either a
 * persistent grid of 2, 3, 4 or 6 workgroups per CU that pull items from a
 * device queue, or one workgroup per item.  The launches and the per-mesh
 * reductions are captured once in a HIP graph and replayed.  Each group's
 * launch form and workgroup size (128 or 256) are picked on the first call
 * by timing the candidates on a strided sample of its work items (about
 * 1.5e8 pairs; cached per shape class for the process).  Results are
 * bitwise those of nlfem_assemble on each mesh alone.                        */
typedef struct nlfem_batch nlfem_batch;

/* meshes[n], params[n] (HOST arrays of structs; the mesh arrays they point to
 * follow mem_kind).  All params must use the same precision, cap sampling and
 * keying.  With 8 or more meshes the symbolic phases run on 4 host threads,
 * each with a stream of its own (the call waits for ctx's stream first and
 * returns when all are done); the plans' memory is ctx's either way, and
 * after a successful build ctx's cache keeps the threads' temporaries.  If
 * any mesh fails, every plan built so far and the threads' temporaries are
 * freed and the first failure is returned (message via nlfem_last_error).     */
nlfem_status nlfem_batch_create(nlfem_ctx *ctx, int32_t n, const nlfem_mesh *meshes,
                                const nlfem_params *params, nlfem_batch **batch);
nlfem_status nlfem_batch_info(const nlfem_batch *batch, int32_t i, int64_t *n_free, int64_t *nnz_ff,
                              int64_t *nnz_fc, int64_t pair_counts[5]);
/* f_qp[i], g_nodal[i]: DEVICE pointers per mesh (as in nlfem_assemble; the
 * host arrays f_qp / g_nodal may themselves be NULL for all-zero inputs).
 * Outputs stay in the batch's device buffers (nlfem_batch_system).  The
 * graph is re-captured when a g pointer changes.                              */
nlfem_status nlfem_batch_assemble(nlfem_batch *batch, const double *const *f_qp,
                                  const double *const *g_nodal);
/* DEVICE pointers to mesh i's assembled system, owned by the batch.           */
nlfem_status nlfem_batch_system(const nlfem_batch *batch, int32_t i, const int64_t **ff_row_ptr,
                                const int32_t **ff_col, const double **ff_val,
                                const int64_t **fc_row_ptr, const int32_t **fc_col,
                                const double **fc_val, const double **rhs,
                                const int32_t **free_to_vertex);
/* Chosen workgroup size of the group with the most pairs and its number of
 * workgroups (the persistent grid, or its number of work items), the
 * integration time of the chosen shapes on the tuning samples summed over
 * the groups, and the time of the last graph replay (milliseconds, HIP
 * events).                                                                   */
nlfem_status nlfem_batch_tuning(const nlfem_batch *batch, int32_t *block, int32_t *grid,
                                double *tuned_integrate_ms, double *last_graph_ms);
/* Pins the launch shape of every group instead of the autotuner's choice:
 * workgroup size block (128 or 256) and a persistent grid of wg_per_cu
 * workgroups per CU, or wg_per_cu = 0 for one workgroup per work item
 * ((block / 64) * wg_per_cu <= 12).  Takes effect on the next
 * nlfem_batch_assemble, which captures its graph again; results do not
 * depend on the shape.                                                       */
nlfem_status nlfem_batch_set_launch(nlfem_batch *batch, int32_t block, int32_t wg_per_cu);
nlfem_status nlfem_batch_destroy(nlfem_batch *batch);

/* Device kernel timing of the last nlfem_assemble / nlfem_plan_create on the
 * plan, measured with HIP events on the context's stream (milliseconds):
 * times[0] plan total, [1] classify, [2] local vertex sets + row lists + CSR
 * pattern, [3] integrate, [4] row assembly (inner-element terms, rows, rhs),
 * [5] assemble total.                                                        */
nlfem_status nlfem_plan_timings(const nlfem_plan *plan, double times[6]);

/* ---- serving -----------------------------------------------------------------
 * A request loop for assemble-and-solve requests of different meshes,
 * horizons, sample counts and precisions (the solve of the linear system of
 * Sec. 4.3 for each request, by CG).  The server owns n_slots slots, each a
 * worker thread with its own HIP stream, and one device memory pool of
 * pool_bytes (0 = half of the free device memory) from which every request
 * takes all of its device buffers: mesh, pair lists, workspace, CSR and CG
 * vectors stay on the device for the whole request.  Queued requests are
 * admitted in arrival order, first fit, when a slot is free and their
 * estimated footprint fits in the pool next to the running ones (a request
 * passed over 16 times holds the others back until it fits).  The estimate is
 * a geometric model of the plan's sizes, scaled down by the largest measured
 * peak / model ratio of finished requests with a similar model value (plus
 * 15 %), never above the model.  A request that
 * runs out of pool memory is re-queued with its measured need, and fails with
 * NLFEM_E_OOM only when it does not fit alone.  Requests overlap on the
 * device (continuous batching); each request's solution is bitwise the one it
 * gets alone.                                                                  */
typedef struct nlfem_server nlfem_server;

typedef struct {
    double rtol;       /* CG stop: ||r||_2 <= rtol ||b||_2                       */
    int32_t max_iter;  /* CG iteration cap; 0 = 10 n_free + 100                  */
} nlfem_solve_params;

typedef struct {
    int32_t state;            /* 0 queued, 1 running, 2 done, 3 failed                      */
    int32_t status;           /* nlfem_status of a finished request                          */
    int64_t n_free, nnz_ff, nnz_fc;
    int64_t pair_counts[5];   /* as nlfem_plan_info                                          */
    int32_t cg_iters;
    int32_t attempts;         /* admissions (more than 1 after an out-of-pool re-queue)      */
    double cg_rel_residual;
    double queue_s, plan_s, assemble_s, solve_s;  /* arrival->admission, plan, assembly, CG + copy */
    double latency_s;         /* arrival (submit) -> solution in host memory                 */
    size_t est_bytes;         /* admission estimate of the device footprint                  */
    size_t peak_bytes;        /* measured peak of pool memory held by the request            */
} nlfem_request_info;

typedef struct {
    int64_t queued, running, done, failed;
    int32_t max_running;      /* most requests that ran at once                              */
    int32_t n_slots;
    size_t pool_bytes, pool_used, pool_peak;
} nlfem_server_counters;

nlfem_status nlfem_server_create(int device, int32_t n_slots, size_t pool_bytes, nlfem_server **server);
/* Queues one request.  mesh arrays (mem_kind must be 0), params.outer_mask,
 * f_qp [n_tets][4] and g_nodal [n_vertices] are HOST memory (f_qp, g_nodal
 * NULL = 0), copied before the call returns.  solve NULL = rtol 1e-10,
 * default cap.  The arrival time of the request is the time of the call.      */
nlfem_status nlfem_server_submit(nlfem_server *server, const nlfem_mesh *mesh, const nlfem_params *params,
                                 const double *f_qp, const double *g_nodal, const nlfem_solve_params *solve,
                                 uint64_t *ticket);
nlfem_status nlfem_server_poll(nlfem_server *server, uint64_t ticket, nlfem_request_info *info);
/* Waits until the request is done or failed (timeout_s < 0: no limit), then
 * fills info (NULL allowed).                                                  */
nlfem_status nlfem_server_wait(nlfem_server *server, uint64_t ticket, double timeout_s,
                               nlfem_request_info *info);
/* Copies a finished request's solution x [n_free] and free_to_vertex [n_free]
 * (HOST, either NULL to skip) and forgets the request.                        */
nlfem_status nlfem_server_take(nlfem_server *server, uint64_t ticket, double *x, int32_t *free_to_vertex);
nlfem_status nlfem_server_stats(nlfem_server *server, nlfem_server_counters *stats);
/* Message of the last failed request (owned by the server).                  */
const char *nlfem_server_last_error(nlfem_server *server);
/* Drops queued requests, waits for the running ones, frees the pool.         */
nlfem_status nlfem_server_destroy(nlfem_server *server);

#ifdef __cplusplus
}
#endif
#endif /* NLFEM_H */
