/* Runs the serial oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure: built and run by tests/test_sanitizers.py).  The
 * oracle source is compiled into this translation unit.
 *
 * Input: a binary case file (little endian), repeated until end of file:
 *   int64 V, K; double delta, psi; int32 N; uint64 seed;
 *   int32 strategy, cap_sampling, keying, g_degree, has_mask;
 *   double coords[V][3]; int32 tets[K][4]; uint8 vertex_free[V];
 *   double f_qp[K][4]; double g_nodal[V]; uint8 mask[K] (if has_mask);
 *   double g_coef[(g_degree + 1)^3] (if g_degree >= 0).
 * Each case is assembled; the free rows of A must sum to zero against their
 * scale (constant kernel, A 1 = 0), A_ff must be symmetric, and the CG must
 * run.  Prints one line per case and "ok" at the end; any sanitizer report
 * ends the process with a nonzero status. */
#include "../../oracle/nlfem_oracle.c"

#include <stdio.h>

static int rd(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(3);
    }
    return p;
}

static double entry(const or_system *S, int64_t r, int32_t c) {
    for (int64_t e = S->ff_row_ptr[r]; e < S->ff_row_ptr[r + 1]; ++e)
        if (S->ff_col[e] == c) return S->ff_val[e];
    return 0.0;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s cases.bin\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int ncase = 0;
    for (;;) {
        int64_t V, K;
        if (!rd(f, &V, 8)) break;
        or_problem P;
        memset(&P, 0, sizeof P);
        int32_t N, strategy, caps, keying, gdeg, has_mask;
        uint64_t seed;
        double delta, psi;
        if (!rd(f, &K, 8) || !rd(f, &delta, 8) || !rd(f, &psi, 8) || !rd(f, &N, 4) || !rd(f, &seed, 8) ||
            !rd(f, &strategy, 4) || !rd(f, &caps, 4) || !rd(f, &keying, 4) || !rd(f, &gdeg, 4) || !rd(f, &has_mask, 4))
            return 2;
        double *coords = xmalloc((size_t)V * 24);
        int32_t *tets = xmalloc((size_t)K * 16);
        uint8_t *vfree = xmalloc((size_t)V);
        double *fqp = xmalloc((size_t)K * 32);
        double *g = xmalloc((size_t)V * 8);
        uint8_t *mask = has_mask ? xmalloc((size_t)K) : NULL;
        const int64_t ncoef = gdeg >= 0 ? (int64_t)(gdeg + 1) * (gdeg + 1) * (gdeg + 1) : 0;
        double *coef = gdeg >= 0 ? xmalloc((size_t)ncoef * 8) : NULL;
        if (!rd(f, coords, (size_t)V * 24) || !rd(f, tets, (size_t)K * 16) || !rd(f, vfree, (size_t)V) ||
            !rd(f, fqp, (size_t)K * 32) || !rd(f, g, (size_t)V * 8) || (mask && !rd(f, mask, (size_t)K)) ||
            (coef && !rd(f, coef, (size_t)ncoef * 8)))
            return 2;
        P.n_vertices = V;
        P.n_tets = K;
        P.coords = coords;
        P.tets = tets;
        P.vertex_free = vfree;
        P.delta = delta;
        P.psi = psi;
        P.mc_samples = N;
        P.seed = seed;
        P.outer_mask = mask;
        P.f_qp = fqp;
        P.g_nodal = g;
        P.strategy = strategy;
        P.cap_sampling = caps;
        P.g_degree = gdeg >= 0 ? gdeg : 0;
        P.g_coef = coef;
        P.keying = keying;
        or_system S;
        memset(&S, 0, sizeof S);
        const int rc = or_assemble(&P, &S);
        if (rc != 0) {
            fprintf(stderr, "case %d: or_assemble returned %d\n", ncase, rc);
            return 1;
        }
        double worst_sum = 0.0, worst_sym = 0.0;
        for (int64_t r = 0; r < S.n_free; ++r) {
            double tot = 0.0, mag = 0.0, asym = 0.0;
            for (int64_t e = S.ff_row_ptr[r]; e < S.ff_row_ptr[r + 1]; ++e) {
                tot += S.ff_val[e];
                mag = fmax(mag, fabs(S.ff_val[e]));
                asym = fmax(asym, fabs(entry(&S, S.ff_col[e], (int32_t)r) - S.ff_val[e]));
            }
            for (int64_t e = S.fc_row_ptr[r]; e < S.fc_row_ptr[r + 1]; ++e) {
                tot += S.fc_val[e];
                mag = fmax(mag, fabs(S.fc_val[e]));
            }
            if (mag > 0.0) {
                worst_sum = fmax(worst_sum, fabs(tot) / mag);
                worst_sym = fmax(worst_sym, asym / mag);
            }
        }
        double *x = xmalloc((size_t)S.n_free * 8);
        memset(x, 0, (size_t)S.n_free * 8);
        int32_t iters = 0;
        double relres = 0.0;
        (void)or_cg(S.n_free, S.ff_row_ptr, S.ff_col, S.ff_val, S.rhs, x, 1e-10, 1000, &iters, &relres);
        printf("case %d: V=%lld K=%lld free=%lld nnz=%lld row sums %.2e symmetry %.2e cg %d its\n", ncase,
               (long long)V, (long long)K, (long long)S.n_free, (long long)S.nnz_ff, worst_sum, worst_sym, iters);
        /* every pair's local matrix is symmetric and annihilates constants,
         * so A is symmetric and A 1 = 0 up to rounding, for every strategy */
        if (worst_sum > 1e-10 || worst_sym > 1e-10) {
            fprintf(stderr, "case %d: invariant failed\n", ncase);
            return 1;
        }
        or_system_free(&S);
        free(x);
        free(coords);
        free(tets);
        free(vfree);
        free(fqp);
        free(g);
        free(mask);
        free(coef);
        ++ncase;
    }
    fclose(f);
    if (ncase == 0) return 2;
    printf("ok\n");
    return 0;
}
