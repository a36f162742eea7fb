/*
 * nlfem_oracle.c -- serial FP64 reference ("oracle") for the fullcaps assembly
 * of the 3D P1 nonlocal Poisson stiffness matrix and load vector.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never calls into it, and it
 * shares no code, header or constant table with the HIP library.
 *
 * What it computes (paper: Chen, Ma & Zhang, "High performance implementation
 * of 3D FEM for nonlocal Poisson problem with different ball approximation
 * strategies"):
 *   - the linear system of eq. (modified_linear): A_h restricted to the free
 *     rows and split into the free x free block A_ff and the free x
 *     constrained block A_fc, and the load vector  b = F_h - A_fc g;
 *   - the outer integral by the 4-point degree-2 rule on every T_Omega tet
 *     (Sec. 4.2.1, "Nocaps with Gauss Quadrature Rules");
 *   - the inner integral over the approximate ball B_{delta,h}(p) built by
 *     the fullcaps strategy (Sec. 4.2.2, Algorithm "construction of fullcaps"):
 *     inside tets by the 4-point rule, cut tets by the 4-point rule on the
 *     subdivision T_I of conv(I u P) (Def. "simplex's dividing strategy")
 *     plus Monte Carlo over the fullcap (E - U_I) n B_delta(p);
 *   - the per-(point, element) Tuples/Pairs of the main assembly algorithm
 *     (Sec. 4.3), reduced by sort + reduce as the paper's Sec. 4.4 describes;
 *   - an unpreconditioned FP64 conjugate-gradient solve.
 * The ball query is brute force over every tet of the mesh (the definition
 * of the ball; the paper's breadth-first search visits the same set when the
 * intersecting tets are face-connected).
 *
 * Readings of points the paper leaves open are listed in the design notes and
 * repeated at the functions that take them.  All arithmetic is IEEE double,
 * compiled with -ffp-contract=off; fma() appears only where written out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OUT 0
#define OR_IN 1
#define OR_CUT0 2 /* CUT with n_in inside vertices is OR_CUT0 + n_in */

/* ------------------------------------------------------------------------ */
/* 4-point degree-2 rule on a tetrahedron (Sec. 4.2.1: the same rule is used for
 * the outer and the inner integrals).  Barycentric node r has weight 1/4 and
 * coordinates alpha on vertex r, beta on the others, with
 * alpha = (5 + 3 sqrt 5)/20, beta = (5 - sqrt 5)/20.                          */
static double g_alpha, g_beta;
static int g_init;
static void rule_init(void) {
    if (g_init) return;
    g_alpha = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
    g_beta = (5.0 - sqrt(5.0)) / 20.0;
    g_init = 1;
}
static double rule(int r, int l) { return r == l ? g_alpha : g_beta; }

void or_rule_constants(double *alpha, double *beta) {
    rule_init();
    *alpha = g_alpha;
    *beta = g_beta;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with multipliers
 * 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.   */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform point in a tetrahedron as barycentric coordinates: the spacings of
 * three sorted uniform integers on [0, 2^21) are a Dirichlet(1,1,1,1) draw
 * (Devroye, Non-Uniform Random Variate Generation, spacings of uniform order
 * statistics).  One Philox call (key = seed) feeds two samples: sample s even
 * uses the top 21 bits of words 0..2; sample s odd uses the top 21 bits of
 * word 3 and two 21-bit fields made of the low bits of words 0,1 and 2,3.  All
 * lambdas are exact multiples of 2^-21.
 * Counters (the paper leaves the sampling open, Sec. 4.2.2):
 *   pair keying    (keying 0): (q, m, floor(s/2), 0) -- N samples of their
 *                  own for every (outer point, element) pair;
 *   element keying (keying 1): (m, floor(s/2), 0, 1) -- N samples per element
 *                  E_m, the same points of E_m for every outer point q.      */
static void sort3(uint32_t *a, uint32_t *b, uint32_t *c) {
    uint32_t t;
    if (*a > *b) { t = *a; *a = *b; *b = t; }
    if (*b > *c) { t = *b; *b = *c; *c = t; }
    if (*a > *b) { t = *a; *a = *b; *b = t; }
}

void or_sample_lambda_keyed(uint64_t seed, int keying, uint32_t q, uint32_t m, uint32_t s, double lam[4]) {
    uint32_t ctr[4] = {q, m, s >> 1, 0u};
    if (keying == 1) {
        ctr[0] = m;
        ctr[1] = s >> 1;
        ctr[2] = 0u;
        ctr[3] = 1u;
    }
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint32_t u0, u1, u2;
    if ((s & 1u) == 0u) {
        u0 = w[0] >> 11; u1 = w[1] >> 11; u2 = w[2] >> 11;
    } else {
        u0 = w[3] >> 11;
        u1 = ((w[0] & 0x7FFu) << 10) | (w[1] & 0x3FFu);
        u2 = ((w[2] & 0x7FFu) << 10) | (w[3] & 0x3FFu);
    }
    sort3(&u0, &u1, &u2);
    const double sc = 1.0 / 2097152.0; /* 2^-21 */
    lam[0] = (double)u0 * sc;
    lam[1] = (double)(u1 - u0) * sc;
    lam[2] = (double)(u2 - u1) * sc;
    lam[3] = (double)(2097152u - u2) * sc;
}

void or_sample_lambda(uint64_t seed, uint32_t q, uint32_t m, uint32_t s, double lam[4]) {
    or_sample_lambda_keyed(seed, 0, q, m, s, lam);
}

/* ------------------------------------------------------------------------ */
/* small geometry                                                            */
static double dot3(const double a[3], const double b[3]) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* det[b-a, c-a, d-a] expanded along the first row */
static double orient3(const double a[3], const double b[3], const double c[3], const double d[3]) {
    double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
    double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
    double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
    return bx * (cy * dz - cz * dy) - by * (cx * dz - cz * dx) + bz * (cx * dy - cy * dx);
}

/* Tet volume |det(X1-X0, X2-X0, X3-X0)| / 6 (either orientation accepted). */
static double tet_volume(const double X[4][3]) {
    return fabs(orient3(X[0], X[1], X[2], X[3])) / 6.0;
}

/* Squared distance from p to the closed triangle (a, b, c), by the Voronoi
 * region method for the closest point on a triangle (Ericson, Real-Time
 * Collision Detection, Sec. 5.1.5).                                          */
static double dist2_point_triangle(const double p[3], const double a[3], const double b[3],
                                   const double c[3]) {
    double ab[3], ac[3], ap[3], bp[3], cp[3], q[3];
    for (int i = 0; i < 3; ++i) {
        ab[i] = b[i] - a[i];
        ac[i] = c[i] - a[i];
        ap[i] = p[i] - a[i];
    }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int i = 0; i < 3; ++i) q[i] = a[i];
        goto done;
    }
    for (int i = 0; i < 3; ++i) bp[i] = p[i] - b[i];
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) {
        for (int i = 0; i < 3; ++i) q[i] = b[i];
        goto done;
    }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
        goto done;
    }
    for (int i = 0; i < 3; ++i) cp[i] = p[i] - c[i];
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) {
        for (int i = 0; i < 3; ++i) q[i] = c[i];
        goto done;
    }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
        goto done;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
        goto done;
    }
    {
        double denom = 1.0 / ((va + vb) + vc);
        double v = vb * denom, w = vc * denom;
        for (int i = 0; i < 3; ++i) q[i] = (a[i] + ab[i] * v) + ac[i] * w;
    }
done:;
    double e[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return dot3(e, e);
}

/* Closed tet vs open ball, for a tet with no vertex inside the ball: they meet
 * iff p lies in the closed tet or some face is closer than delta.           */
static int tet_meets_ball_no_vertex_inside(const double X[4][3], const double p[3], double d2) {
    double o = orient3(X[0], X[1], X[2], X[3]);
    double o0 = orient3(p, X[1], X[2], X[3]);
    double o1 = orient3(X[0], p, X[2], X[3]);
    double o2 = orient3(X[0], X[1], p, X[3]);
    double o3 = orient3(X[0], X[1], X[2], p);
    int inside = (o > 0.0) ? (o0 >= 0.0 && o1 >= 0.0 && o2 >= 0.0 && o3 >= 0.0)
                           : (o0 <= 0.0 && o1 <= 0.0 && o2 <= 0.0 && o3 <= 0.0);
    if (inside) return 1;
    if (dist2_point_triangle(p, X[1], X[2], X[3]) < d2) return 1;
    if (dist2_point_triangle(p, X[0], X[2], X[3]) < d2) return 1;
    if (dist2_point_triangle(p, X[0], X[1], X[3]) < d2) return 1;
    if (dist2_point_triangle(p, X[0], X[1], X[2]) < d2) return 1;
    return 0;
}

/* Classification of tet X against the open ball B_delta(p)
 * (Def. "simplex's dividing strategy"): a vertex is inside iff its squared
 * distance is < delta^2 (open ball).  4 inside -> IN; 1..3 -> CUT(n_in); 0 ->
 * CUT(0) when the tet still meets the ball (the definition notes that an
 * all-vertices-outside tet may intersect the ball, and the fullcaps
 * construction samples such a tet whole), otherwise OUT.                     */
static int classify(const double X[4][3], const double p[3], double d2, double r2[4]) {
    int n_in = 0;
    for (int l = 0; l < 4; ++l) {
        double dx = X[l][0] - p[0], dy = X[l][1] - p[1], dz = X[l][2] - p[2];
        r2[l] = (dx * dx + dy * dy) + dz * dz;
        if (r2[l] < d2) ++n_in;
    }
    if (n_in == 4) return OR_IN;
    if (n_in > 0) return OR_CUT0 + n_in;
    return tet_meets_ball_no_vertex_inside(X, p, d2) ? OR_CUT0 : OR_OUT;
}

/* Ball approximation strategies (Sec. 4.1: the approximate ball B_delta,h(p)
 * as a set of whole elements or element pieces):
 *   FULLCAPS   elements inside, T_I of the cut ones, and the fullcaps by
 *              Monte Carlo (Sec. 4.2.2; the default);
 *   NOCAPS     elements inside and T_I of the cut ones (Def. nocaps): the
 *              fullcaps dropped, CUT(0) elements contribute nothing;
 *   OVERLAP    every element that meets the ball, whole;
 *   INSIDE     only the elements wholly inside the ball, whole;
 *   BARYCENTER the elements whose barycenter lies in the ball, whole.
 * The last three map a pair to IN (whole element, 4-point rule) or OUT.    */
#define OR_FULLCAPS 0
#define OR_NOCAPS 1
#define OR_OVERLAP 2
#define OR_INSIDE 3
#define OR_BARYCENTER 4

/* barycenter c = ((X_0 + X_1) + (X_2 + X_3)) / 4 in the open ball */
static int barycenter_inside(const double X[4][3], const double p[3], double d2) {
    double r2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        double c = ((X[0][i] + X[1][i]) + (X[2][i] + X[3][i])) * 0.25;
        double d = c - p[i];
        r2 = (i == 0) ? d * d : r2 + d * d;
    }
    return r2 < d2;
}

/* class of a pair under a strategy, from its fullcaps class */
static int strategy_class(int cls, const double X[4][3], const double p[3], double d2, int strategy) {
    switch (strategy) {
    case OR_NOCAPS: return cls == OR_CUT0 ? OR_OUT : cls;
    case OR_OVERLAP: return cls == OR_OUT ? OR_OUT : OR_IN;
    case OR_INSIDE: return cls == OR_IN ? OR_IN : OR_OUT;
    case OR_BARYCENTER: return barycenter_inside(X, p, d2) ? OR_IN : OR_OUT;
    default: return cls;
    }
}

/* ------------------------------------------------------------------------ */
/* Cut-tet geometry in barycentric (lambda) space of the inner tet.          */
typedef struct {
    int n_in;
    int I[4], O[4];
    double t[4][4];       /* t[a][b]: edge a->b meets the sphere at X_a + t (X_b - X_a) */
    int n_sub;
    double sub[3][4][4];  /* subtet s, vertex r, barycentric component l */
    double subdet[3];     /* |det| of subtet s in lambda space (physical vol = |E| * subdet) */
    int n_planes;
    double plane[2][4];   /* U_I = E n {lambda : plane[i] . lambda >= 0 for all i} */
    int split;            /* n_in = 2: 1 or 2 (which diagonal of the interior quad) */
} cutgeom;

/* det of (b1-b0, b2-b0, b3-b0) over barycentric components 1..3 */
static double det3_bary(const double b0[4], const double b1[4], const double b2[4], const double b3[4]) {
    double ax = b1[1] - b0[1], ay = b1[2] - b0[2], az = b1[3] - b0[3];
    double bx = b2[1] - b0[1], by = b2[2] - b0[2], bz = b2[3] - b0[3];
    double cx = b3[1] - b0[1], cy = b3[2] - b0[2], cz = b3[3] - b0[3];
    return ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
}

static double det3m(double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                    double c1, double c2) {
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

/* Linear functional c on R^4 vanishing on the barycentric points Q1, Q2, Q3
 * (cofactors of the first row of det[x; Q1; Q2; Q3]), oriented so that the
 * sum of its values at the inside vertices is non-negative.                 */
static void plane_through(const double *Q1, const double *Q2, const double *Q3, const cutgeom *g,
                          double c[4]) {
    c[0] = det3m(Q1[1], Q1[2], Q1[3], Q2[1], Q2[2], Q2[3], Q3[1], Q3[2], Q3[3]);
    c[1] = -det3m(Q1[0], Q1[2], Q1[3], Q2[0], Q2[2], Q2[3], Q3[0], Q3[2], Q3[3]);
    c[2] = det3m(Q1[0], Q1[1], Q1[3], Q2[0], Q2[1], Q2[3], Q3[0], Q3[1], Q3[3]);
    c[3] = -det3m(Q1[0], Q1[1], Q1[2], Q2[0], Q2[1], Q2[2], Q3[0], Q3[1], Q3[2]);
    double s = 0.0;
    for (int i = 0; i < g->n_in; ++i) s = s + c[g->I[i]];
    if (s < 0.0)
        for (int l = 0; l < 4; ++l) c[l] = -c[l];
}

static void unit(int a, double e[4]) {
    for (int l = 0; l < 4; ++l) e[l] = (l == a) ? 1.0 : 0.0;
}

static void edge_point(const cutgeom *g, int a, int b, double e[4]) {
    for (int l = 0; l < 4; ++l) e[l] = 0.0;
    e[a] = 1.0 - g->t[a][b];
    e[b] = g->t[a][b];
}

static void set_sub(cutgeom *g, int s, const double *v0, const double *v1, const double *v2,
                    const double *v3) {
    for (int l = 0; l < 4; ++l) {
        g->sub[s][0][l] = v0[l];
        g->sub[s][1][l] = v1[l];
        g->sub[s][2][l] = v2[l];
        g->sub[s][3][l] = v3[l];
    }
}

/* Builds T_I = subdivision of U_I = conv(I u P) and the half-space form of U_I
 * (fullcaps construction, Sec. 4.2.2).  P holds the m (4-m) edge points where
 * the sphere crosses the edges joining inside and outside vertices.
 *  - edge point: X_a + t (X_b - X_a) with |.| = delta, the root in (0,1] of
 *    A t^2 + 2 B t + C = 0, A = |X_b-X_a|^2, B = (X_a-p).(X_b-X_a),
 *    C = |X_a-p|^2 - delta^2 < 0, taken in the cancellation-free form;
 *  - n_in = 1: U_I is the corner tet at the inside vertex;
 *  - n_in = 3: U_I is the prism E minus the corner at the outside vertex,
 *    split into 3 tets;
 *  - n_in = 2: U_I is conv{a, b, P_ac, P_ad, P_bc, P_bd}, a prism whose
 *    interior quad (P_ac, P_ad, P_bd, P_bc) is skew; of the two diagonal
 *    choices the convex hull is the one with the larger volume (tie: the
 *    first, diagonal P_ac-P_bd).                                            */
static void cut_geometry(const double X[4][3], const double p[3], double d2, const double r2[4],
                         cutgeom *g) {
    int ni = 0, no = 0;
    for (int l = 0; l < 4; ++l) {
        if (r2[l] < d2) g->I[ni++] = l;
        else g->O[no++] = l;
    }
    g->n_in = ni;
    g->n_sub = 0;
    g->n_planes = 0;
    g->split = 0;
    memset(g->t, 0, sizeof g->t);
    for (int i = 0; i < ni; ++i) {
        int a = g->I[i];
        double ea[3] = {X[a][0] - p[0], X[a][1] - p[1], X[a][2] - p[2]};
        for (int j = 0; j < no; ++j) {
            int b = g->O[j];
            double dv[3] = {X[b][0] - X[a][0], X[b][1] - X[a][1], X[b][2] - X[a][2]};
            double A = dot3(dv, dv);
            double B = dot3(ea, dv);
            double C = r2[a] - d2;
            double s = sqrt(B * B - A * C);
            double t = (B <= 0.0) ? (s - B) / A : (-C) / (B + s);
            if (t > 1.0) t = 1.0;
            g->t[a][b] = t;
        }
    }
    if (ni == 1) {
        int a = g->I[0], b = g->O[0], c = g->O[1], d = g->O[2];
        double A[4], Pb[4], Pc[4], Pd[4];
        unit(a, A);
        edge_point(g, a, b, Pb);
        edge_point(g, a, c, Pc);
        edge_point(g, a, d, Pd);
        set_sub(g, 0, A, Pb, Pc, Pd);
        g->n_sub = 1;
        plane_through(Pb, Pc, Pd, g, g->plane[0]);
        g->n_planes = 1;
    } else if (ni == 3) {
        int a = g->I[0], b = g->I[1], c = g->I[2], d = g->O[0];
        double A[4], B[4], C[4], A1[4], B1[4], C1[4];
        unit(a, A); unit(b, B); unit(c, C);
        edge_point(g, a, d, A1);
        edge_point(g, b, d, B1);
        edge_point(g, c, d, C1);
        set_sub(g, 0, A, B, C, C1);
        set_sub(g, 1, A, B, B1, C1);
        set_sub(g, 2, A, A1, B1, C1);
        g->n_sub = 3;
        plane_through(A1, B1, C1, g, g->plane[0]);
        g->n_planes = 1;
    } else if (ni == 2) {
        int a = g->I[0], b = g->I[1], c = g->O[0], d = g->O[1];
        double A[4], B[4], C[4], A1[4], B1[4], C1[4];
        unit(a, A);
        edge_point(g, a, c, B);
        edge_point(g, a, d, C);
        unit(b, A1);
        edge_point(g, b, c, B1);
        edge_point(g, b, d, C1);
        double v1 = fabs(det3_bary(A, B, C, C1)) + fabs(det3_bary(A, B, B1, C1)) +
                    fabs(det3_bary(A, A1, B1, C1));
        double v2 = fabs(det3_bary(A, B, C, B1)) + fabs(det3_bary(A, C, B1, C1)) +
                    fabs(det3_bary(A, A1, B1, C1));
        if (v1 >= v2) {
            set_sub(g, 0, A, B, C, C1);
            set_sub(g, 1, A, B, B1, C1);
            set_sub(g, 2, A, A1, B1, C1);
            plane_through(B, C, C1, g, g->plane[0]);
            plane_through(B, B1, C1, g, g->plane[1]);
            g->split = 1;
        } else {
            set_sub(g, 0, A, B, C, B1);
            set_sub(g, 1, A, C, B1, C1);
            set_sub(g, 2, A, A1, B1, C1);
            plane_through(B, C, B1, g, g->plane[0]);
            plane_through(C, B1, C1, g, g->plane[1]);
            g->split = 2;
        }
        g->n_sub = 3;
        g->n_planes = 2;
    }
    for (int s = 0; s < g->n_sub; ++s)
        g->subdet[s] = fabs(det3_bary(g->sub[s][0], g->sub[s][1], g->sub[s][2], g->sub[s][3]));
}

/* Value of the plane functional c at lambda: c . lambda summed in vertex order,
 * ((c_0 lambda_0 + c_1 lambda_1) + c_2 lambda_2) + c_3 lambda_3.              */
static double plane_value(const double c[4], const double lam[4]) {
    return ((c[0] * lam[0] + c[1] * lam[1]) + c[2] * lam[2]) + c[3] * lam[3];
}

/* ------------------------------------------------------------------------ */
/* Inner-integral node enumeration for one (outer point, inner tet) pair.
 * Every node is (lambda, weight): lambda = barycentric coordinates of the
 * node in the inner tet, weight = its share of the inner integral's measure.
 *  - IN:  the 4-point rule on E_m (weights |E_m|/4);
 *  - CUT: the 4-point rule on every subtet of T_I (weights |sub|/4), then the
 *         accepted Monte Carlo samples: N uniform points of E_m, each with
 *         weight |E_m|/N, accepted iff |y - p| < delta and y not in U_I
 *         (the fullcap (E - U_I) n B_delta(p); CUT(0) has U_I empty).       */
typedef struct {
    const double (*X)[3];
    double p[3];
    double d2;
    double vol;
    int cls;
    double r2[4];
    cutgeom g;
    int N;
    int caps; /* 1: the fullcaps Monte Carlo term is part of the pair */
    int cap_sampling; /* 1: for n_in >= 1 the caps are sampled on E - U_I (cap_region) */
    int keying;       /* 0: samples per (point, element) pair, 1: per element (or_sample_lambda_keyed) */
    uint64_t seed;
    uint32_t q, m;
    /* near-tie report (optional, may be NULL): samples whose decision lies
     * within the rounding band of the sample test, and the sum of their weights */
    int64_t *ties;
    double *tie_w;
    /* per-sample record for tests (optional, may be NULL, indexed by s):
     * |y - p|^2, accepted, near tie */
    double *rec_rr;
    int8_t *rec_acc, *rec_tie;
} pairctx;

typedef void (*node_fn)(void *user, const double lam[4], double w, int is_mc);

/* ------------------------------------------------------------------------ */
/* The cap region E - U_I (closure of E minus the inner polytope), sampled
 * instead of the whole E when cap sampling is on (Sec. 4.2.2 leaves the
 * sampling of the caps open).  U_I = E n {planes >= 0}; the first outside
 * vertex o = O[0] lies strictly outside every plane (each plane separates the
 * inside from the outside vertices along the edges it cuts), and a point of E
 * outside U_I lies outside at least one plane, so the segment from o to it
 * stays outside U_I: E - U_I is star-shaped from o.  The cones from o over its
 * boundary faces that do not contain o therefore tile it:
 *  - n_in = 3 (inside a0 < a1 < a2): one face, the cut triangle; the corner
 *    tet (o; P_a0o, P_a1o, P_a2o);
 *  - n_in = 1 (inside a, outside o < c < d): the cut triangle (P_ao, P_ac,
 *    P_ad) and the quad (c, d, P_ad, P_ac) left of face a c d, halved on its
 *    diagonal c-P_ad: (o; P_ao, P_ac, P_ad), (o; c, d, P_ad), (o; c, P_ad, P_ac);
 *  - n_in = 2 (inside a < b, outside o < d): the triangle (d, P_ad, P_bd) left
 *    of face a b d and the two triangles of U_I's inner quad on the diagonal
 *    U_I uses; P_ao-P_bd: (o; d, P_ad, P_bd), (o; P_ao, P_ad, P_bd),
 *    (o; P_ao, P_bo, P_bd); P_ad-P_bo: (o; d, P_ad, P_bd), (o; P_ao, P_ad, P_bo),
 *    (o; P_ad, P_bo, P_bd).
 * P_xy is the sphere crossing on the edge from inside x to outside y.  A
 * point's offset from p is X_a - p for a vertex and (X_x - p) + t (X_y - X_x)
 * (one FMA) for a crossing.  The corner tet's volume is
 * |E| (1 - t_0)(1 - t_1)(1 - t_2), a cone tet's |E| |det of its rows|.       */
typedef struct {
    int a, b; /* vertex a (b < 0) or the crossing on edge a -> b */
} rpoint;

typedef struct {
    int n;               /* sub-tets: 1 (n_in = 3) or 3 (n_in = 1, 2) */
    double row[3][4][4]; /* sub-tet j, point r (r = 0: o), barycentric component */
    double e[3][4][3];   /* point minus p */
    double vol[3];
} capregion;

static void region_point(const pairctx *c, rpoint q, double row[4], double e[3]) {
    if (q.b < 0) {
        unit(q.a, row);
        for (int i = 0; i < 3; ++i) e[i] = c->X[q.a][i] - c->p[i];
    } else {
        const double t = c->g.t[q.a][q.b];
        edge_point(&c->g, q.a, q.b, row);
        for (int i = 0; i < 3; ++i) e[i] = fma(t, c->X[q.b][i] - c->X[q.a][i], c->X[q.a][i] - c->p[i]);
    }
}

static int cap_region(const pairctx *c, capregion *r) {
    const cutgeom *g = &c->g;
    const int o = g->O[0];
    rpoint V[3][4];
    for (int j = 0; j < 3; ++j) V[j][0] = (rpoint){o, -1};
    if (g->n_in == 3) {
        r->n = 1;
        for (int l = 0; l < 3; ++l) V[0][1 + l] = (rpoint){g->I[l], o};
    } else if (g->n_in == 1) {
        const int a = g->I[0], cc = g->O[1], d = g->O[2];
        r->n = 3;
        V[0][1] = (rpoint){a, o};   V[0][2] = (rpoint){a, cc};  V[0][3] = (rpoint){a, d};
        V[1][1] = (rpoint){cc, -1}; V[1][2] = (rpoint){d, -1};  V[1][3] = (rpoint){a, d};
        V[2][1] = (rpoint){cc, -1}; V[2][2] = (rpoint){a, d};   V[2][3] = (rpoint){a, cc};
    } else if (g->n_in == 2) {
        const int a = g->I[0], b = g->I[1], d = g->O[1];
        r->n = 3;
        V[0][1] = (rpoint){d, -1}; V[0][2] = (rpoint){a, d}; V[0][3] = (rpoint){b, d};
        if (g->split == 1) {
            V[1][1] = (rpoint){a, o}; V[1][2] = (rpoint){a, d}; V[1][3] = (rpoint){b, d};
            V[2][1] = (rpoint){a, o}; V[2][2] = (rpoint){b, o}; V[2][3] = (rpoint){b, d};
        } else {
            V[1][1] = (rpoint){a, o}; V[1][2] = (rpoint){a, d}; V[1][3] = (rpoint){b, o};
            V[2][1] = (rpoint){a, d}; V[2][2] = (rpoint){b, o}; V[2][3] = (rpoint){b, d};
        }
    } else {
        return 0;
    }
    for (int j = 0; j < r->n; ++j)
        for (int q = 0; q < 4; ++q) region_point(c, V[j][q], r->row[j][q], r->e[j][q]);
    if (r->n == 1) {
        double rho = 1.0;
        for (int l = 0; l < 3; ++l) {
            const double t = g->t[g->I[l]][o];
            rho = (l == 0) ? 1.0 - t : rho * (1.0 - t);
        }
        r->vol[0] = c->vol * rho;
    } else {
        for (int j = 0; j < 3; ++j)
            r->vol[j] = c->vol * fabs(det3_bary(r->row[j][0], r->row[j][1], r->row[j][2], r->row[j][3]));
    }
    return 1;
}


static void visit_nodes(const pairctx *c, node_fn fn, void *user) {
    if (c->cls == OR_OUT) return;
    if (c->cls == OR_IN) {
        double w = c->vol * 0.25;
        for (int r = 0; r < 4; ++r) {
            double lam[4];
            for (int l = 0; l < 4; ++l) lam[l] = rule(r, l);
            fn(user, lam, w, 0);
        }
        return;
    }
    const cutgeom *g = &c->g;
    for (int s = 0; s < g->n_sub; ++s) {
        double w = (c->vol * g->subdet[s]) * 0.25;
        for (int r = 0; r < 4; ++r) {
            double lam[4];
            for (int l = 0; l < 4; ++l)
                lam[l] = ((rule(r, 0) * g->sub[s][0][l] + rule(r, 1) * g->sub[s][1][l]) +
                          rule(r, 2) * g->sub[s][2][l]) + rule(r, 3) * g->sub[s][3][l];
            fn(user, lam, w, 0);
        }
    }
    if (!c->caps) return;
    /* Sampling region: the whole E (samples in U_I rejected), or, with cap
     * sampling on and n_in >= 1, E - U_I itself (cap_region), no U_I test.
     * Sub-tet j of n takes the samples s with floor(j N / n) <= s <
     * floor((j + 1) N / n), N_j of them (N >= 3), each of weight |T_j| / N_j;
     * a sample's coordinates mu in T_j give its barycentrics in E as
     * lambda = sum_r mu_r row(T_j, r).
     *
     * Sample test (the fullcap (E - U_I) n B_delta(p), Sec. 4.2.2), in the plain
     * form: y - p = ((mu_0 e_0 + mu_1 e_1) + mu_2 e_2) + mu_3 e_3 per
     * coordinate, e_l = (vertex l of the sampled tet) - p; accepted iff
     * (y - p).(y - p) < delta^2 and lambda is not in U_I.
     *
     * Near ties.  A sample whose decision another correct evaluation order of
     * the same test could reverse is reported (ties, tie_w): the ball test when
     * |(y - p).(y - p) - delta^2| <= 2^-40 E2, E2 = max_l |e_l|^2, and the U_I
     * test when some plane value h_i has |h_i| <= 2^-40 sum_l |c_il| while the
     * other planes hold within their bands and the ball test does not reject
     * beyond its band.  2^-40 is 8192 units of the last place: above the
     * rounding error of any evaluation of these few-term sums (a few dozen
     * roundings of terms no larger than E2, or sum |c|).                    */
    capregion R;
    const int region = c->cap_sampling && cap_region(c, &R);
    const int nb = region ? R.n : 1;
    const double band = 0x1p-40;
    double tau_p[2] = {0.0, 0.0};
    for (int i = 0; i < g->n_planes; ++i)
        tau_p[i] = band * (((fabs(g->plane[i][0]) + fabs(g->plane[i][1])) + fabs(g->plane[i][2])) +
                           fabs(g->plane[i][3]));
    for (int j = 0; j < nb; ++j) {
        double e[4][3];
        for (int l = 0; l < 4; ++l)
            for (int i = 0; i < 3; ++i) e[l][i] = region ? R.e[j][l][i] : c->X[l][i] - c->p[i];
        double E2 = 0.0;
        for (int l = 0; l < 4; ++l) {
            const double r = dot3(e[l], e[l]);
            if (r > E2) E2 = r;
        }
        const double tau_b = band * E2;
        const int s0 = (int)(((int64_t)j * c->N) / nb), s1 = (int)(((int64_t)(j + 1) * c->N) / nb);
        const double wmc = (region ? R.vol[j] : c->vol) / (double)(s1 - s0);
        for (int s = s0; s < s1; ++s) {
            double mu[4];
            or_sample_lambda_keyed(c->seed, c->keying, c->q, c->m, (uint32_t)s, mu);
            double d[3];
            for (int i = 0; i < 3; ++i) d[i] = ((mu[0] * e[0][i] + mu[1] * e[1][i]) + mu[2] * e[2][i]) + mu[3] * e[3][i];
            const double rr = dot3(d, d);
            int acc = rr < c->d2;
            int tie = fabs(rr - c->d2) <= tau_b;
            double lam[4];
            if (region) {
                for (int v = 0; v < 4; ++v)
                    lam[v] = ((mu[0] * R.row[j][0][v] + mu[1] * R.row[j][1][v]) + mu[2] * R.row[j][2][v]) +
                             mu[3] * R.row[j][3][v];
            } else {
                for (int v = 0; v < 4; ++v) lam[v] = mu[v];
                if (g->n_planes > 0) {
                    int inU = 1, near = 0, hold = 1;
                    for (int i = 0; i < g->n_planes; ++i) {
                        const double h = plane_value(g->plane[i], mu);
                        if (!(h >= 0.0)) inU = 0;
                        if (fabs(h) <= tau_p[i]) near = 1;
                        if (h < -tau_p[i]) hold = 0;
                    }
                    if (inU) acc = 0;
                    if (near && hold && rr < c->d2 + tau_b) tie = 1;
                }
            }
            if (c->rec_rr) c->rec_rr[s] = rr;
            if (c->rec_acc) c->rec_acc[s] = (int8_t)acc;
            if (c->rec_tie) c->rec_tie[s] = (int8_t)tie;
            if (tie) {
                if (c->ties) *c->ties += 1;
                if (c->tie_w) *c->tie_w += wmc;
            }
            if (acc) fn(user, lam, wmc, 1);
        }
    }
}

/* Moments of the pair: S0 = sum w, S1_j = sum w lam_j, S2_ij = sum w lam_i
 * lam_j (upper triangle 00,01,02,03,11,12,13,22,23,33).  The deterministic
 * nodes are summed one by one; the Monte Carlo part is summed per block of
 * equal weight (exact dyadic counts for the whole element) and each block
 * scaled by its weight once.                                         */
typedef struct {
    double det[15];
    double mc[15];   /* the current block of Monte Carlo nodes (one weight) */
    double wmc;      /* that weight */
    double done[15]; /* earlier blocks, scaled */
    int nmc;
} momacc;

static void mom_node(void *user, const double lam[4], double w, int is_mc) {
    momacc *a = (momacc *)user;
    if (is_mc) {
        if (a->nmc > 0 && w != a->wmc) {
            for (int k = 0; k < 15; ++k) a->done[k] += a->wmc * a->mc[k];
            memset(a->mc, 0, sizeof a->mc);
        }
        a->nmc++;
        a->wmc = w;
        a->mc[0] += 1.0;
        for (int j = 0; j < 4; ++j) a->mc[1 + j] += lam[j];
        int k = 5;
        for (int i = 0; i < 4; ++i)
            for (int j = i; j < 4; ++j) a->mc[k++] += lam[i] * lam[j];
    } else {
        a->det[0] += w;
        for (int j = 0; j < 4; ++j) a->det[1 + j] += w * lam[j];
        int k = 5;
        for (int i = 0; i < 4; ++i)
            for (int j = i; j < 4; ++j) a->det[k++] += (w * lam[i]) * lam[j];
    }
}

static void pair_setup(pairctx *c, const double X[4][3], const double p[3], double delta, int N,
                       uint64_t seed, uint32_t q, uint32_t m, int strategy, int cap_sampling, int keying) {
    memset(c, 0, sizeof *c);
    c->X = X;
    for (int i = 0; i < 3; ++i) c->p[i] = p[i];
    c->d2 = delta * delta;
    c->vol = tet_volume(X);
    c->N = N;
    c->seed = seed;
    c->q = q;
    c->m = m;
    c->cls = strategy_class(classify(X, p, c->d2, c->r2), X, p, c->d2, strategy);
    c->caps = strategy == OR_FULLCAPS;
    c->cap_sampling = cap_sampling;
    c->keying = keying;
    if (c->cls >= OR_CUT0) cut_geometry(X, p, c->d2, c->r2, &c->g);
}

static void pair_moments(const pairctx *c, double S[15]) {
    momacc a;
    memset(&a, 0, sizeof a);
    visit_nodes(c, mom_node, &a);
    for (int k = 0; k < 15; ++k) S[k] = a.det[k] + (a.done[k] + a.wmc * a.mc[k]);
}

/* ------------------------------------------------------------------------ */
/* outer quadrature point k of tet X: p = sum_l rule(k,l) X_l                 */
static void outer_point(const double X[4][3], int k, double p[3]) {
    rule_init();
    for (int i = 0; i < 3; ++i)
        p[i] = ((rule(k, 0) * X[0][i] + rule(k, 1) * X[1][i]) + rule(k, 2) * X[2][i]) +
               rule(k, 3) * X[3][i];
}

static void load_tet(const double *coords, const int32_t *tets, int64_t m, double X[4][3]) {
    for (int l = 0; l < 4; ++l) {
        int32_t v = tets[4 * m + l];
        for (int i = 0; i < 3; ++i) X[l][i] = coords[3 * (int64_t)v + i];
    }
}

/* ---- public per-point / per-pair entry points (for the tests) ------------ */

void or_outer_point(const double *coords, const int32_t *tets, int64_t n, int k, double p[3]) {
    double X[4][3];
    load_tet(coords, tets, n, X);
    outer_point(X, k, p);
}

/* classes of every tet against the ball around p (codes: 0 OUT, 1 IN, 2+n_in CUT) */
void or_classify_point(const double *coords, const int32_t *tets, int64_t n_tets, double delta,
                       const double p[3], int8_t *cls) {
    double d2 = delta * delta;
    for (int64_t m = 0; m < n_tets; ++m) {
        double X[4][3], r2[4];
        load_tet(coords, tets, m, X);
        cls[m] = (int8_t)classify(X, p, d2, r2);
    }
}

/* moments of pair (outer point q = 4 n + k, inner tet m) with sample keying
 * `keying`; returns the class.  ties (may be NULL) gets the number of its
 * Monte Carlo samples whose decision lies within the rounding band.        */
int or_pair_moments_keyed(const double *coords, const int32_t *tets, int64_t n, int k, int64_t m,
                          double delta, int N, uint64_t seed, int strategy, int cap_sampling, int keying,
                          double S[15], int32_t *ties) {
    double Xn[4][3], Xm[4][3], p[3];
    rule_init();
    load_tet(coords, tets, n, Xn);
    outer_point(Xn, k, p);
    load_tet(coords, tets, m, Xm);
    pairctx c;
    pair_setup(&c, Xm, p, delta, N, seed, (uint32_t)(4 * n + k), (uint32_t)m, strategy, cap_sampling, keying);
    int64_t nt = 0;
    c.ties = &nt;
    for (int i = 0; i < 15; ++i) S[i] = 0.0;
    if (c.cls != OR_OUT) pair_moments(&c, S);
    if (ties) *ties = (int32_t)nt;
    return c.cls;
}

int or_pair_moments(const double *coords, const int32_t *tets, int64_t n, int k, int64_t m,
                    double delta, int N, uint64_t seed, int strategy, int cap_sampling, double S[15]) {
    return or_pair_moments_keyed(coords, tets, n, k, m, delta, N, seed, strategy, cap_sampling, 0, S, NULL);
}

/* all pairs of one outer point against every tet: class + moments (+ near-tie
 * counts per tet when ties is not NULL) */
void or_point_moments_keyed(const double *coords, const int32_t *tets, int64_t n_tets, int64_t n, int k,
                            double delta, int N, uint64_t seed, int strategy, int cap_sampling, int keying,
                            int8_t *cls, double *S /*[n_tets][15]*/, int32_t *ties /*[n_tets]*/) {
    for (int64_t m = 0; m < n_tets; ++m)
        cls[m] = (int8_t)or_pair_moments_keyed(coords, tets, n, k, m, delta, N, seed, strategy, cap_sampling,
                                               keying, S + 15 * m, ties ? ties + m : NULL);
}

void or_point_moments(const double *coords, const int32_t *tets, int64_t n_tets, int64_t n, int k,
                      double delta, int N, uint64_t seed, int strategy, int cap_sampling, int8_t *cls,
                      double *S /*[n_tets][15]*/) {
    or_point_moments_keyed(coords, tets, n_tets, n, k, delta, N, seed, strategy, cap_sampling, 0, cls, S, NULL);
}

/* Monte Carlo samples of one pair, for tests: per sample s, |y - p|^2 as the
 * sample test evaluates it, whether it was accepted, and whether it is a near
 * tie.  Returns the class (samples are recorded for CUT pairs under fullcaps
 * only; other entries are left untouched).                                  */
int or_pair_samples(const double *coords, const int32_t *tets, int64_t n, int k, int64_t m, double delta,
                    int N, uint64_t seed, int cap_sampling, int keying, double *rr, int8_t *acc, int8_t *tie) {
    double Xn[4][3], Xm[4][3], p[3];
    rule_init();
    load_tet(coords, tets, n, Xn);
    outer_point(Xn, k, p);
    load_tet(coords, tets, m, Xm);
    pairctx c;
    pair_setup(&c, Xm, p, delta, N, seed, (uint32_t)(4 * n + k), (uint32_t)m, OR_FULLCAPS, cap_sampling, keying);
    c.rec_rr = rr;
    c.rec_acc = acc;
    c.rec_tie = tie;
    if (c.cls >= OR_CUT0) {
        double S[15];
        pair_moments(&c, S);
    }
    return c.cls;
}

/* cut geometry of a pair, for geometric pins: returns n_in (or -1 if not CUT) */
int or_pair_geometry(const double *coords, const int32_t *tets, int64_t n, int k, int64_t m,
                     double delta, double t_out[16], double sub_out[48], double subvol_out[3],
                     double plane_out[8], int *n_sub, int *n_planes, int *split) {
    double Xn[4][3], Xm[4][3], p[3];
    rule_init();
    load_tet(coords, tets, n, Xn);
    outer_point(Xn, k, p);
    load_tet(coords, tets, m, Xm);
    pairctx c;
    pair_setup(&c, Xm, p, delta, 1, 0, 0, 0, OR_FULLCAPS, 0, 0);
    if (c.cls < OR_CUT0) return -1;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) t_out[4 * a + b] = c.g.t[a][b];
    for (int s = 0; s < 3; ++s)
        for (int r = 0; r < 4; ++r)
            for (int l = 0; l < 4; ++l) sub_out[16 * s + 4 * r + l] = c.g.sub[s][r][l];
    for (int s = 0; s < 3; ++s) subvol_out[s] = s < c.g.n_sub ? c.vol * c.g.subdet[s] : 0.0;
    for (int i = 0; i < 2; ++i)
        for (int l = 0; l < 4; ++l) plane_out[4 * i + l] = c.g.plane[i][l];
    *n_sub = c.g.n_sub;
    *n_planes = c.g.n_planes;
    *split = c.g.split;
    return c.g.n_in;
}

/* the cap region E - U_I of pair (q = 4 n + k, m): its sub-tets' barycentric
 * rows [3][4][4] and volumes; returns the number of sub-tets (0 for CUT(0)),
 * -1 when the pair is not cut */
int or_cap_region(const double *coords, const int32_t *tets, int64_t n, int k, int64_t m, double delta,
                  double row_out[48], double vol_out[3]) {
    double Xn[4][3], Xm[4][3], p[3];
    rule_init();
    load_tet(coords, tets, n, Xn);
    outer_point(Xn, k, p);
    load_tet(coords, tets, m, Xm);
    pairctx c;
    pair_setup(&c, Xm, p, delta, 3, 0, 0, 0, OR_FULLCAPS, 1, 0);
    if (c.cls < OR_CUT0) return -1;
    capregion R;
    if (!cap_region(&c, &R)) return 0;
    for (int j = 0; j < R.n; ++j) {
        vol_out[j] = R.vol[j];
        for (int r = 0; r < 4; ++r)
            for (int l = 0; l < 4; ++l) row_out[16 * j + 4 * r + l] = R.row[j][r][l];
    }
    return R.n;
}

/* ------------------------------------------------------------------------ */
/* Assembly (Sec. 4.3, main algorithm).                                      */
typedef struct {
    int64_t n_vertices, n_tets;
    const double *coords;
    const int32_t *tets;
    const uint8_t *vertex_free;
    const uint8_t *tet_region; /* optional: 1 = T_Omega, 0 = T_Omega_I */
    double delta, psi;
    int32_t mc_samples;
    uint64_t seed;
    const uint8_t *outer_mask; /* optional */
    const double *f_qp;        /* optional [n_tets][4] */
    const double *g_nodal;     /* optional [n_vertices] */
    int32_t strategy;          /* OR_FULLCAPS .. OR_BARYCENTER */
    int32_t cap_sampling;      /* 1: caps of n_in >= 1 sampled on E - U_I (N >= 3) */
    int32_t g_degree;          /* per-axis degree of g_coef */
    const double *g_coef;      /* optional: g as a tensor polynomial -> the right-hand side of
                                  eq. F1.5 with g itself inside the inner integrals of eq. Fh */
    int32_t keying;            /* 0: Monte Carlo samples per (point, element) pair, 1: per element */
} or_problem;

typedef struct {
    int64_t n_free, nnz_ff, nnz_fc;
    int64_t *ff_row_ptr;
    int32_t *ff_col;
    double *ff_val;
    int64_t *fc_row_ptr;
    int32_t *fc_col;
    double *fc_val;
    double *rhs;
    int32_t *free_to_vertex;
    int64_t pair_counts[5]; /* IN, CUT0, CUT1, CUT2, CUT3 */
    /* Near ties of the Monte Carlo sample test (see visit_nodes): their
     * number, and per free row the most any matrix entry of the row
     * (tie_allow) or the right-hand side entry (tie_allow_rhs) can move if
     * another evaluation order decides every near tie the other way: a sample
     * of weight w changes K_uv of its pair by at most f_m |psi| w_k w, since
     * |a_u a_v| <= 1.                                                       */
    int64_t near_ties;
    double *tie_allow;
    double *tie_allow_rhs;
} or_system;

typedef struct {
    int32_t row, col;
    int64_t seq;
    double val;
} tuple_t;

typedef struct {
    tuple_t *a;
    int64_t n, cap, seq;
} tuples;

static int tuple_cmp(const void *x, const void *y) {
    const tuple_t *a = (const tuple_t *)x, *b = (const tuple_t *)y;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
    return 0;
}

/* sort by (row, col, emission order) and add up equal keys in emission order */
static void tuples_reduce(tuples *T) {
    if (T->n == 0) return;
    qsort(T->a, (size_t)T->n, sizeof(tuple_t), tuple_cmp);
    int64_t w = 0;
    for (int64_t i = 1; i < T->n; ++i) {
        if (T->a[i].row == T->a[w].row && T->a[i].col == T->a[w].col) {
            T->a[w].val = T->a[w].val + T->a[i].val;
        } else {
            T->a[++w] = T->a[i];
        }
    }
    T->n = w + 1;
}

static int tuples_push(tuples *T, int32_t row, int32_t col, double val) {
    if (T->n == T->cap) {
        tuples_reduce(T);
        if (T->n > T->cap / 2) {
            int64_t nc = T->cap * 2;
            tuple_t *na = (tuple_t *)realloc(T->a, (size_t)nc * sizeof(tuple_t));
            if (!na) return -1;
            T->a = na;
            T->cap = nc;
        }
    }
    T->a[T->n].row = row;
    T->a[T->n].col = col;
    T->a[T->n].seq = T->seq++;
    T->a[T->n].val = val;
    T->n++;
    return 0;
}

/* Local matrix of one pair in the literal form of the paper: for every node
 * y with weight w, a_u(y) = phi_(m,u)(y) - phi_(n,u)(p) for u in V_n u V_m,
 * and local[u][v] += w a_u a_v.                                             */
typedef struct {
    int nu;
    int32_t U[8];
    int jm[8]; /* local index in E_m or -1 */
    double c[8]; /* phi_(n,u)(p): the outer rule row, 0 if u not in E_n */
    double L[8][8];
} localmat;

static void local_node(void *user, const double lam[4], double w, int is_mc) {
    (void)is_mc;
    localmat *M = (localmat *)user;
    double a[8];
    for (int u = 0; u < M->nu; ++u) {
        double yv = M->jm[u] >= 0 ? lam[M->jm[u]] : 0.0;
        a[u] = yv - M->c[u];
    }
    for (int u = 0; u < M->nu; ++u)
        for (int v = 0; v < M->nu; ++v) M->L[u][v] += (w * a[u]) * a[v];
}

/* g(y) = sum over a, b, c in 0..deg of coef[a + n1 (b + n1 c)] y1^a y2^b y3^c,
 * n1 = deg + 1, summed monomial by monomial */
static double gpoly_value(const double *coef, int deg, const double y[3]) {
    int n1 = deg + 1;
    double s = 0.0;
    for (int c = 0; c <= deg; ++c)
        for (int b = 0; b <= deg; ++b)
            for (int a = 0; a <= deg; ++a) {
                double mono = 1.0;
                for (int e = 0; e < a; ++e) mono *= y[0];
                for (int e = 0; e < b; ++e) mono *= y[1];
                for (int e = 0; e < c; ++e) mono *= y[2];
                s += coef[a + n1 * (b + n1 * c)] * mono;
            }
    return s;
}

/* inner integral over the pair's nodes of 1 (s0) and of g (gint); a node's
 * point is y = sum_l lambda_l X_l */
typedef struct {
    const double (*X)[3];
    const double *coef;
    int deg;
    double s0, gint;
} ginner;

static void g_node(void *user, const double lam[4], double w, int is_mc) {
    (void)is_mc;
    ginner *a = (ginner *)user;
    double y[3];
    for (int i = 0; i < 3; ++i)
        y[i] = ((lam[0] * a->X[0][i] + lam[1] * a->X[1][i]) + lam[2] * a->X[2][i]) + lam[3] * a->X[3][i];
    a->s0 += w;
    a->gint += w * gpoly_value(a->coef, a->deg, y);
}

static int validate(const or_problem *P) {
    if (!P || P->n_vertices < 0 || P->n_tets < 0) return 1;
    if (!(P->delta > 0.0) || P->mc_samples < 1) return 1;
    if (P->strategy < OR_FULLCAPS || P->strategy > OR_BARYCENTER) return 1;
    if (P->cap_sampling != 0 && P->cap_sampling != 1) return 1;
    if (P->cap_sampling == 1 && P->mc_samples < 3) return 1;
    if (P->keying != 0 && P->keying != 1) return 1;
    if (P->g_coef && (P->g_degree < 0 || P->g_degree > 4 || P->cap_sampling != 0)) return 1;
    if (P->n_tets > 0 && (!P->coords || !P->tets || !P->vertex_free)) return 1;
    for (int64_t i = 0; i < 4 * P->n_tets; ++i)
        if (P->tets[i] < 0 || P->tets[i] >= P->n_vertices) return 2;
    return 0;
}

void or_system_free(or_system *S) {
    if (!S) return;
    free(S->ff_row_ptr); free(S->ff_col); free(S->ff_val);
    free(S->fc_row_ptr); free(S->fc_col); free(S->fc_val);
    free(S->rhs); free(S->free_to_vertex);
    free(S->tie_allow); free(S->tie_allow_rhs);
    memset(S, 0, sizeof *S);
}

static int is_outer(const or_problem *P, const uint8_t *region, int64_t n) {
    return region[n] && (!P->outer_mask || P->outer_mask[n]);
}

/* Returns 0 on success, 1 invalid argument, 2 invalid mesh, 3 out of memory. */
int or_assemble(const or_problem *P, or_system *S) {
    memset(S, 0, sizeof *S);
    int rc = validate(P);
    if (rc) return rc;
    rule_init();
    const int64_t V = P->n_vertices, K = P->n_tets;
    uint8_t *region = (uint8_t *)malloc((size_t)(K > 0 ? K : 1));
    int32_t *free_id = (int32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int32_t));
    if (!region || !free_id) { free(region); free(free_id); return 3; }
    int64_t nf = 0;
    for (int64_t v = 0; v < V; ++v) free_id[v] = P->vertex_free[v] ? (int32_t)nf++ : -1;
    /* T_Omega: given, or the tets with at least one free vertex */
    for (int64_t m = 0; m < K; ++m) {
        int anyfree = 0;
        for (int l = 0; l < 4; ++l) anyfree |= P->vertex_free[P->tets[4 * m + l]] ? 1 : 0;
        region[m] = P->tet_region ? (P->tet_region[m] ? 1 : 0) : (uint8_t)anyfree;
        if (!region[m] && anyfree) { free(region); free(free_id); return 2; }
        double X[4][3];
        load_tet(P->coords, P->tets, m, X);
        if (!(tet_volume(X) > 0.0)) { free(region); free(free_id); return 2; }
    }
    S->n_free = nf;
    S->rhs = (double *)calloc((size_t)(nf > 0 ? nf : 1), sizeof(double));
    S->free_to_vertex = (int32_t *)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(int32_t));
    S->tie_allow = (double *)calloc((size_t)(nf > 0 ? nf : 1), sizeof(double));
    S->tie_allow_rhs = (double *)calloc((size_t)(nf > 0 ? nf : 1), sizeof(double));
    tuples T = {0};
    T.cap = 1 << 22;
    T.a = (tuple_t *)malloc((size_t)T.cap * sizeof(tuple_t));
    if (!S->rhs || !S->free_to_vertex || !S->tie_allow || !S->tie_allow_rhs || !T.a) { free(T.a); free(region); free(free_id); or_system_free(S); return 3; }
    for (int64_t v = 0; v < V; ++v)
        if (free_id[v] >= 0) S->free_to_vertex[free_id[v]] = (int32_t)v;

    const double d2 = P->delta * P->delta;
    for (int64_t n = 0; n < K; ++n) {
        if (!is_outer(P, region, n)) continue;
        double Xn[4][3];
        load_tet(P->coords, P->tets, n, Xn);
        const double wk = tet_volume(Xn) / 4.0;
        for (int k = 0; k < 4; ++k) {
            double p[3];
            outer_point(Xn, k, p);
            /* Pairs: (i, phi_i(p) f(p) w) once per outer point */
            if (P->f_qp) {
                double fp = P->f_qp[4 * n + k];
                for (int j = 0; j < 4; ++j) {
                    int32_t u = P->tets[4 * n + j];
                    if (free_id[u] >= 0) S->rhs[free_id[u]] += (wk * rule(k, j)) * fp;
                }
            }
            for (int64_t m = 0; m < K; ++m) {
                double Xm[4][3];
                load_tet(P->coords, P->tets, m, Xm);
                pairctx c;
                memset(&c, 0, sizeof c);
                c.X = Xm;
                for (int i = 0; i < 3; ++i) c.p[i] = p[i];
                c.d2 = d2;
                c.cls = strategy_class(classify(Xm, p, d2, c.r2), Xm, p, d2, P->strategy);
                if (c.cls == OR_OUT) continue;
                c.vol = tet_volume(Xm);
                c.N = P->mc_samples;
                c.caps = P->strategy == OR_FULLCAPS;
                c.cap_sampling = P->cap_sampling;
                c.keying = P->keying;
                c.seed = P->seed;
                c.q = (uint32_t)(4 * n + k);
                c.m = (uint32_t)m;
                if (c.cls >= OR_CUT0) cut_geometry(Xm, p, d2, c.r2, &c.g);
                S->pair_counts[c.cls == OR_IN ? 0 : 1 + (c.cls - OR_CUT0)]++;
                localmat M;
                memset(&M, 0, sizeof M);
                for (int j = 0; j < 4; ++j) {
                    M.U[j] = P->tets[4 * n + j];
                    M.jm[j] = -1;
                    M.c[j] = rule(k, j);
                }
                M.nu = 4;
                for (int j = 0; j < 4; ++j) {
                    int32_t v = P->tets[4 * m + j];
                    int found = -1;
                    for (int u = 0; u < M.nu; ++u)
                        if (M.U[u] == v) found = u;
                    if (found < 0) {
                        found = M.nu++;
                        M.U[found] = v;
                        M.c[found] = 0.0;
                    }
                    M.jm[found] = j;
                }
                int64_t nties = 0;
                double tie_w = 0.0;
                c.ties = &nties;
                c.tie_w = &tie_w;
                visit_nodes(&c, local_node, &M);
                c.ties = NULL;
                c.tie_w = NULL;
                /* Tuples (i, j, a w) with psi and the kernel factor of the
                 * inner element: 1 on T_Omega (the W term), 2 on T_Omega_I
                 * (the N term together with the Omega_I coupling moved to the
                 * right-hand side through the nodal constraint values).     */
                double fm = region[m] ? 1.0 : 2.0;
                double scale = (P->psi * fm) * wk;
                if (nties > 0) {
                    /* rows of the pair's free vertices; the right-hand side moves
                     * through A_fc g over the pair's constrained vertices */
                    double gsum = 0.0;
                    for (int v = 0; v < M.nu; ++v)
                        if (free_id[M.U[v]] < 0 && P->g_nodal) gsum += fabs(P->g_nodal[M.U[v]]);
                    const double da = fabs(scale) * tie_w;
                    for (int u = 0; u < M.nu; ++u) {
                        int32_t fu = free_id[M.U[u]];
                        if (fu < 0) continue;
                        S->tie_allow[fu] += da;
                        S->tie_allow_rhs[fu] += da * gsum;
                    }
                    S->near_ties += nties;
                }
                if (P->g_coef) {
                    /* eq. F1.5 with F_h of eq. Fh, term by term:
                     * T_Omega inner element: - A_h(phi_j, phi_i) g_j for the
                     *   boundary nodes j, from the W term of eq. notreplaced;
                     * T_Omega_I inner element: + 2 psi w phi_i(p) int g (the
                     *   F_h term), and - the N term 2 psi w phi_j(p) phi_i(p)
                     *   int 1 times g_j for the boundary nodes j of E_n.       */
                    if (region[m]) {
                        for (int u = 0; u < M.nu; ++u) {
                            int32_t fu = free_id[M.U[u]];
                            if (fu < 0) continue;
                            for (int v = 0; v < M.nu; ++v)
                                if (free_id[M.U[v]] < 0 && P->g_nodal)
                                    S->rhs[fu] -= (scale * M.L[u][v]) * P->g_nodal[M.U[v]];
                        }
                    } else {
                        ginner gi = {c.X, P->g_coef, P->g_degree, 0.0, 0.0};
                        visit_nodes(&c, g_node, &gi);
                        for (int u = 0; u < 4; ++u) {
                            int32_t fu = free_id[M.U[u]];
                            if (fu < 0) continue;
                            double pu = (2.0 * P->psi) * (wk * M.c[u]);
                            S->rhs[fu] += pu * gi.gint;
                            for (int v = 0; v < 4; ++v)
                                if (free_id[M.U[v]] < 0 && P->g_nodal)
                                    S->rhs[fu] -= ((pu * M.c[v]) * gi.s0) * P->g_nodal[M.U[v]];
                        }
                    }
                }
                for (int u = 0; u < M.nu; ++u) {
                    int32_t fu = free_id[M.U[u]];
                    if (fu < 0) continue;
                    for (int v = 0; v < M.nu; ++v)
                        if (tuples_push(&T, fu, M.U[v], scale * M.L[u][v])) {
                            free(T.a); free(region); free(free_id); or_system_free(S); return 3;
                        }
                }
            }
        }
    }
    tuples_reduce(&T);
    /* split rows into the free and constrained column blocks */
    S->ff_row_ptr = (int64_t *)calloc((size_t)nf + 1, sizeof(int64_t));
    S->fc_row_ptr = (int64_t *)calloc((size_t)nf + 1, sizeof(int64_t));
    int64_t nff = 0, nfc = 0;
    for (int64_t i = 0; i < T.n; ++i) {
        if (free_id[T.a[i].col] >= 0) { nff++; S->ff_row_ptr[T.a[i].row + 1]++; }
        else { nfc++; S->fc_row_ptr[T.a[i].row + 1]++; }
    }
    for (int64_t r = 0; r < nf; ++r) {
        S->ff_row_ptr[r + 1] += S->ff_row_ptr[r];
        S->fc_row_ptr[r + 1] += S->fc_row_ptr[r];
    }
    S->nnz_ff = nff;
    S->nnz_fc = nfc;
    S->ff_col = (int32_t *)malloc((size_t)(nff > 0 ? nff : 1) * sizeof(int32_t));
    S->ff_val = (double *)malloc((size_t)(nff > 0 ? nff : 1) * sizeof(double));
    S->fc_col = (int32_t *)malloc((size_t)(nfc > 0 ? nfc : 1) * sizeof(int32_t));
    S->fc_val = (double *)malloc((size_t)(nfc > 0 ? nfc : 1) * sizeof(double));
    if (!S->ff_col || !S->ff_val || !S->fc_col || !S->fc_val) {
        free(T.a); free(region); free(free_id); or_system_free(S); return 3;
    }
    int64_t iff = 0, ifc = 0;
    for (int64_t i = 0; i < T.n; ++i) {
        int32_t c = T.a[i].col;
        if (free_id[c] >= 0) { S->ff_col[iff] = free_id[c]; S->ff_val[iff++] = T.a[i].val; }
        else { S->fc_col[ifc] = c; S->fc_val[ifc++] = T.a[i].val; }
    }
    /* b = F_h - A_fc g  (nodal constraint values; the exact-g form was summed above) */
    if (P->g_nodal && !P->g_coef) {
        for (int64_t r = 0; r < nf; ++r) {
            double acc = 0.0;
            for (int64_t e = S->fc_row_ptr[r]; e < S->fc_row_ptr[r + 1]; ++e)
                acc = acc + S->fc_val[e] * P->g_nodal[S->fc_col[e]];
            S->rhs[r] = S->rhs[r] - acc;
        }
    }
    free(T.a);
    free(region);
    free(free_id);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Unpreconditioned conjugate gradient on a CSR matrix (the solve of the main
 * algorithm).  x holds x0 on entry.  Stops when ||r||_2 <= rtol ||b||_2.
 * Returns 0 converged, 4 not converged.                                      */
static void spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, const double *x,
                 double *y) {
    for (int64_t r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) acc = acc + va[e] * x[ci[e]];
        y[r] = acc;
    }
}

static double dotn(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

int or_cg(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, const double *b,
          double *x, double rtol, int32_t max_iter, int32_t *iters, double *relres) {
    *iters = 0;
    double bn = sqrt(dotn(n, b, b));
    if (n == 0 || bn == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        *relres = 0.0;
        return 0;
    }
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *pv = (double *)malloc((size_t)n * sizeof(double));
    double *Ap = (double *)malloc((size_t)n * sizeof(double));
    spmv(n, rp, ci, va, x, Ap);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - Ap[i]; pv[i] = r[i]; }
    double rr = dotn(n, r, r);
    int it = 0, conv = sqrt(rr) <= rtol * bn;
    while (!conv && it < max_iter) {
        spmv(n, rp, ci, va, pv, Ap);
        double alpha = rr / dotn(n, pv, Ap);
        for (int64_t i = 0; i < n; ++i) { x[i] = x[i] + alpha * pv[i]; r[i] = r[i] - alpha * Ap[i]; }
        double rr1 = dotn(n, r, r);
        ++it;
        conv = sqrt(rr1) <= rtol * bn;
        double beta = rr1 / rr;
        for (int64_t i = 0; i < n; ++i) pv[i] = r[i] + beta * pv[i];
        rr = rr1;
    }
    *iters = it;
    *relres = sqrt(rr) / bn;
    free(r); free(pv); free(Ap);
    return conv ? 0 : 4;
}
