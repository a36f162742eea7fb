// Device-side geometry, classification, fullcaps subdivision and Monte Carlo
// sampling for one (outer point, inner tet) pair.
//
// Every floating-point expression is written out in a fixed evaluation order
// and the library is compiled with -ffp-contract=off; fused multiply-adds
// appear only where written as fma().  With IEEE-correct sqrt and division
// this makes classification and sample acceptance bit-reproducible.
#pragma once

#include "common.hpp"

namespace nlfem {

__device__ __forceinline__ double rule_w(int r, int l) { return r == l ? kAlpha : kBeta; }

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

// det[b-a, c-a, d-a], first-row expansion
__device__ __forceinline__ double orient3(const double* a, const double* b, const double* c, const double* d) {
    double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
    double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
    double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
    return bx * (cy * dz - cz * dy) - by * (cx * dz - cz * dx) + bz * (cx * dy - cy * dx);
}

// outer quadrature point k of the tet with vertices X (row-major [4][3])
__device__ __forceinline__ void outer_point(const double* X, int k, double* p) {
    for (int i = 0; i < 3; ++i)
        p[i] = ((rule_w(k, 0) * X[i] + rule_w(k, 1) * X[3 + i]) + rule_w(k, 2) * X[6 + i]) +
               rule_w(k, 3) * X[9 + i];
}

// squared distance from p to the closed triangle (a, b, c): Voronoi-region
// closest point (Ericson, Real-Time Collision Detection, Sec. 5.1.5)
__device__ inline double dist2_tri(const double* p, const double* a, const double* b, const double* c) {
    double ab[3], ac[3], ap[3], q[3];
    for (int i = 0; i < 3; ++i) {
        ab[i] = b[i] - a[i];
        ac[i] = c[i] - a[i];
        ap[i] = p[i] - a[i];
    }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int i = 0; i < 3; ++i) q[i] = a[i];
    } else {
        double bp[3];
        for (int i = 0; i < 3; ++i) bp[i] = p[i] - b[i];
        double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
        if (d3 >= 0.0 && d4 <= d3) {
            for (int i = 0; i < 3; ++i) q[i] = b[i];
        } else {
            double vc = d1 * d4 - d3 * d2;
            if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
                double v = d1 / (d1 - d3);
                for (int i = 0; i < 3; ++i) q[i] = a[i] + v * ab[i];
            } else {
                double cp[3];
                for (int i = 0; i < 3; ++i) cp[i] = p[i] - c[i];
                double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
                if (d6 >= 0.0 && d5 <= d6) {
                    for (int i = 0; i < 3; ++i) q[i] = c[i];
                } else {
                    double vb = d5 * d2 - d1 * d6;
                    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
                        double w = d2 / (d2 - d6);
                        for (int i = 0; i < 3; ++i) q[i] = a[i] + w * ac[i];
                    } else {
                        double va = d3 * d6 - d5 * d4;
                        if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
                            double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
                            for (int i = 0; i < 3; ++i) q[i] = b[i] + w * (c[i] - b[i]);
                        } else {
                            double denom = 1.0 / ((va + vb) + vc);
                            double v = vb * denom, w = vc * denom;
                            for (int i = 0; i < 3; ++i) q[i] = (a[i] + ab[i] * v) + ac[i] * w;
                        }
                    }
                }
            }
        }
    }
    double e[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return dot3(e, e);
}

// closed tet (no vertex inside the open ball) meets the open ball?
__device__ inline bool meets_ball(const double* X, const double* p, double d2) {
    const double *X0 = X, *X1 = X + 3, *X2 = X + 6, *X3 = X + 9;
    double o = orient3(X0, X1, X2, X3);
    double o0 = orient3(p, X1, X2, X3);
    double o1 = orient3(X0, p, X2, X3);
    double o2 = orient3(X0, X1, p, X3);
    double o3 = orient3(X0, X1, X2, p);
    bool inside = (o > 0.0) ? (o0 >= 0.0 && o1 >= 0.0 && o2 >= 0.0 && o3 >= 0.0)
                            : (o0 <= 0.0 && o1 <= 0.0 && o2 <= 0.0 && o3 <= 0.0);
    if (inside) return true;
    if (dist2_tri(p, X1, X2, X3) < d2) return true;
    if (dist2_tri(p, X0, X2, X3) < d2) return true;
    if (dist2_tri(p, X0, X1, X3) < d2) return true;
    if (dist2_tri(p, X0, X1, X2) < d2) return true;
    return false;
}

// Classification against the open ball: 4 vertices inside -> IN, 1..3 ->
// CUT(n_in), none -> CUT(0) if the tet still meets the ball, else OUT.
// A bounding-box distance test first discards tets that are surely apart
// (margin 1e-9 relative, far above rounding), which leaves the result equal
// to the exact test.
__device__ inline int classify(const double* X, const double* p, double d2, double* r2) {
    int nin = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        double dx = X[3 * l] - p[0], dy = X[3 * l + 1] - p[1], dz = X[3 * l + 2] - p[2];
        r2[l] = (dx * dx + dy * dy) + dz * dz;
        nin += (r2[l] < d2) ? 1 : 0;
    }
    if (nin == 4) return C_IN;
    if (nin > 0) return C_CUT0 + nin;
    double bd = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double lo = fmin(fmin(X[i], X[3 + i]), fmin(X[6 + i], X[9 + i]));
        double hi = fmax(fmax(X[i], X[3 + i]), fmax(X[6 + i], X[9 + i]));
        double g = fmax(fmax(lo - p[i], p[i] - hi), 0.0);
        bd += g * g;
    }
    if (bd > d2 * (1.0 + 1e-9)) return C_OUT;
    return meets_ball(X, p, d2) ? C_CUT0 : C_OUT;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t* w) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per multiplier (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
}

// 21-bit uniform triple of sample half h (0: words 0..2 top bits; 1: word 3 top
// bits and the low bits of words 0/1 and 2/3), sorted ascending, as spacings.
__device__ __forceinline__ void lambda_u(const uint32_t* w, int h, uint32_t* L) {
    uint32_t u0, u1, u2;
    if (h == 0) {
        u0 = w[0] >> 11; u1 = w[1] >> 11; u2 = w[2] >> 11;
    } else {
        u0 = w[3] >> 11;
        u1 = ((w[0] & 0x7FFu) << 10) | (w[1] & 0x3FFu);
        u2 = ((w[2] & 0x7FFu) << 10) | (w[3] & 0x3FFu);
    }
    uint32_t a = min(u0, u1), b = max(u0, u1);
    uint32_t b2 = min(b, u2), c = max(b, u2);
    uint32_t a2 = min(a, b2), b3 = max(a, b2);
    L[0] = a2;
    L[1] = b3 - a2;
    L[2] = c - b3;
    L[3] = 2097152u - c;
}

// ---------------------------------------------------------------------------
// Cut-pair geometry in the inner tet's barycentric space.
struct CutGeom {
    int nin;
    int I0, I1, I2;     // inside local vertices (ascending)
    int O0, O1, O2;     // outside local vertices (ascending)
    int nplanes;
    double c0[4], c1[4];  // U_I = E n {c0.l >= 0} [n {c1.l >= 0}]
};

__device__ __forceinline__ double det3m(double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                                        double c1, double c2) {
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

__device__ __forceinline__ double det3_bary(const double* b0, const double* b1, const double* b2, const double* b3) {
    double ax = b1[1] - b0[1], ay = b1[2] - b0[2], az = b1[3] - b0[3];
    double bx = b2[1] - b0[1], by = b2[2] - b0[2], bz = b2[3] - b0[3];
    double cx = b3[1] - b0[1], cy = b3[2] - b0[2], cz = b3[3] - b0[3];
    return ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
}

// functional vanishing on Q1, Q2, Q3; oriented non-negative on the inside vertices
__device__ inline void plane_through(const double* Q1, const double* Q2, const double* Q3, const CutGeom& g,
                                     double* c) {
    c[0] = det3m(Q1[1], Q1[2], Q1[3], Q2[1], Q2[2], Q2[3], Q3[1], Q3[2], Q3[3]);
    c[1] = -det3m(Q1[0], Q1[2], Q1[3], Q2[0], Q2[2], Q2[3], Q3[0], Q3[2], Q3[3]);
    c[2] = det3m(Q1[0], Q1[1], Q1[3], Q2[0], Q2[1], Q2[3], Q3[0], Q3[1], Q3[3]);
    c[3] = -det3m(Q1[0], Q1[1], Q1[2], Q2[0], Q2[1], Q2[2], Q3[0], Q3[1], Q3[2]);
    double s = 0.0;
    s = s + c[g.I0];
    if (g.nin > 1) s = s + c[g.I1];
    if (g.nin > 2) s = s + c[g.I2];
    if (s < 0.0)
        for (int l = 0; l < 4; ++l) c[l] = -c[l];
}

// sphere crossing on edge a (inside) -> b (outside)
__device__ __forceinline__ double edge_t(const double* X, const double* p, double d2, const double* r2, int a, int b) {
    double ea[3] = {X[3 * a] - p[0], X[3 * a + 1] - p[1], X[3 * a + 2] - p[2]};
    double dv[3] = {X[3 * b] - X[3 * a], X[3 * b + 1] - X[3 * a + 1], X[3 * b + 2] - X[3 * a + 2]};
    double A = dot3(dv, dv);
    double B = dot3(ea, dv);
    double C = r2[a] - d2;
    double s = sqrt(B * B - A * C);
    double t = (B <= 0.0) ? (s - B) / A : (-C) / (B + s);
    return t > 1.0 ? 1.0 : t;
}

// Hull points of U_I: (a, b, t) stands for the barycentric point
// (1 - t) e_a + t e_b, or the vertex e_a when b < 0.
struct HullPts {
    int a[6], b[6];
    double t[6];
};

__device__ __forceinline__ void hull_dense(const HullPts& H, int i, double* e) {
    const int a = H.a[i], b = H.b[i];
    const double t = H.t[i];
#pragma unroll
    for (int l = 0; l < 4; ++l) e[l] = (b < 0) ? ((l == a) ? 1.0 : 0.0) : ((l == a) ? 1.0 - t : ((l == b) ? t : 0.0));
}

// Accumulator type for the deterministic subtet rule: T = double or float.
template <typename T>
struct Mom {
    T s[15];
};

// subtet index patterns into the hull point list
//   n_in = 1: {0,1,2,3};  n_in = 3 and n_in = 2 (first diagonal): {0,1,2,5},{0,1,4,5},{0,3,4,5};
//   n_in = 2 (second diagonal): {0,1,2,4},{0,2,4,5},{0,3,4,5}
__device__ __forceinline__ int subtet_vertex(int pattern, int s, int r) {
    // pattern 0: single tet; 1: first prism split; 2: second prism split
    const unsigned P1 = 0x543u << 0;  // unused helper (kept simple below)
    (void)P1;
    if (pattern == 0) return r;
    if (r == 0) return 0;
    if (pattern == 1) {
        if (s == 0) return (r == 1) ? 1 : (r == 2 ? 2 : 5);
        if (s == 1) return (r == 1) ? 1 : (r == 2 ? 4 : 5);
        return (r == 1) ? 3 : (r == 2 ? 4 : 5);
    }
    if (s == 0) return (r == 1) ? 1 : (r == 2 ? 2 : 4);
    if (s == 1) return (r == 1) ? 2 : (r == 2 ? 4 : 5);
    return (r == 1) ? 3 : (r == 2 ? 4 : 5);
}

__device__ __forceinline__ double subtet_absdet(const HullPts& H, int pattern, int s) {
    double v0[4], v1[4], v2[4], v3[4];
    hull_dense(H, subtet_vertex(pattern, s, 0), v0);
    hull_dense(H, subtet_vertex(pattern, s, 1), v1);
    hull_dense(H, subtet_vertex(pattern, s, 2), v2);
    hull_dense(H, subtet_vertex(pattern, s, 3), v3);
    return fabs(det3_bary(v0, v1, v2, v3));
}

// 4-point rule on subtet s of the pattern, weight vol*|det|/4 per node
template <typename T>
__device__ __forceinline__ void subtet_rule(const HullPts& H, int pattern, int s, double vol, Mom<T>& M) {
    double v0[4], v1[4], v2[4], v3[4];
    hull_dense(H, subtet_vertex(pattern, s, 0), v0);
    hull_dense(H, subtet_vertex(pattern, s, 1), v1);
    hull_dense(H, subtet_vertex(pattern, s, 2), v2);
    hull_dense(H, subtet_vertex(pattern, s, 3), v3);
    double det = fabs(det3_bary(v0, v1, v2, v3));
    T w = (T)((vol * det) * 0.25);
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        T xi[4];
#pragma unroll
        for (int l = 0; l < 4; ++l)
            xi[l] = (T)(((rule_w(r, 0) * v0[l] + rule_w(r, 1) * v1[l]) + rule_w(r, 2) * v2[l]) + rule_w(r, 3) * v3[l]);
        M.s[0] += w;
#pragma unroll
        for (int j = 0; j < 4; ++j) M.s[1 + j] += w * xi[j];
        int k = 5;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = i; j < 4; ++j) M.s[k++] += (w * xi[i]) * xi[j];
    }
}

__device__ __forceinline__ void plane_hull(const HullPts& H, int i1, int i2, int i3, const CutGeom& g, double* c) {
    double Q1[4], Q2[4], Q3[4];
    hull_dense(H, i1, Q1);
    hull_dense(H, i2, Q2);
    hull_dense(H, i3, Q3);
    plane_through(Q1, Q2, Q3, g, c);
}

// Build U_I = conv(I u P) (fullcaps construction) as hull points, add the
// 4-point rule on its subdivision T_I to M, and set the half-space form of
// U_I used by the sample test.
//   n_in = 1: corner tet (a; P_ab, P_ac, P_ad), plane (P_ab, P_ac, P_ad)
//   n_in = 3: prism (a, b, c | P_ad, P_bd, P_cd), plane (P_ad, P_bd, P_cd)
//   n_in = 2: prism (a, P_ac, P_ad | b, P_bc, P_bd); its interior quad
//             (P_ac, P_ad, P_bd, P_bc) is split along the diagonal giving the
//             larger (convex) volume, ties to P_ac-P_bd.
template <typename T>
__device__ inline void cut_setup(const double* X, const double* p, double d2, const double* r2, double vol,
                                 CutGeom& g, Mom<T>& M) {
    int I[4], O[4], ni = 0, no = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (r2[l] < d2) I[ni++] = l;
        else O[no++] = l;
    }
    g.nin = ni;
    g.I0 = I[0]; g.I1 = I[1]; g.I2 = I[2];
    g.O0 = O[0]; g.O1 = O[1]; g.O2 = O[2];
    g.nplanes = 0;
    HullPts H;
    int pattern = -1, nsub = 0;
    if (ni == 1) {
        H.a[0] = I[0]; H.b[0] = -1; H.t[0] = 0.0;
        for (int j = 0; j < 3; ++j) {
            H.a[1 + j] = I[0];
            H.b[1 + j] = O[j];
            H.t[1 + j] = edge_t(X, p, d2, r2, I[0], O[j]);
        }
        pattern = 0;
        nsub = 1;
        plane_hull(H, 1, 2, 3, g, g.c0);
        g.nplanes = 1;
    } else if (ni == 3) {
        for (int j = 0; j < 3; ++j) {
            H.a[j] = I[j]; H.b[j] = -1; H.t[j] = 0.0;
            H.a[3 + j] = I[j]; H.b[3 + j] = O[0];
            H.t[3 + j] = edge_t(X, p, d2, r2, I[j], O[0]);
        }
        pattern = 1;
        nsub = 3;
        plane_hull(H, 3, 4, 5, g, g.c0);
        g.nplanes = 1;
    } else if (ni == 2) {
        H.a[0] = I[0]; H.b[0] = -1; H.t[0] = 0.0;
        H.a[1] = I[0]; H.b[1] = O[0]; H.t[1] = edge_t(X, p, d2, r2, I[0], O[0]);
        H.a[2] = I[0]; H.b[2] = O[1]; H.t[2] = edge_t(X, p, d2, r2, I[0], O[1]);
        H.a[3] = I[1]; H.b[3] = -1; H.t[3] = 0.0;
        H.a[4] = I[1]; H.b[4] = O[0]; H.t[4] = edge_t(X, p, d2, r2, I[1], O[0]);
        H.a[5] = I[1]; H.b[5] = O[1]; H.t[5] = edge_t(X, p, d2, r2, I[1], O[1]);
        double v1 = subtet_absdet(H, 1, 0) + subtet_absdet(H, 1, 1) + subtet_absdet(H, 1, 2);
        double v2 = subtet_absdet(H, 2, 0) + subtet_absdet(H, 2, 1) + subtet_absdet(H, 2, 2);
        nsub = 3;
        if (v1 >= v2) {
            pattern = 1;
            plane_hull(H, 1, 2, 5, g, g.c0);
            plane_hull(H, 1, 4, 5, g, g.c1);
        } else {
            pattern = 2;
            plane_hull(H, 1, 2, 4, g, g.c0);
            plane_hull(H, 2, 4, 5, g, g.c1);
        }
        g.nplanes = 2;
    }
#pragma unroll 1
    for (int s = 0; s < nsub; ++s) subtet_rule<T>(H, pattern, s, vol, M);
    // sample test: a missing plane is replaced by one that holds everywhere
    // (c = (1,1,1,1): c.lambda = 1 >= 0), and for n_in = 0 by one that never holds.
    if (g.nplanes < 2) {
        for (int l = 0; l < 4; ++l) g.c1[l] = 1.0;
    }
    if (g.nplanes == 0) {
        for (int l = 0; l < 4; ++l) g.c0[l] = -1.0;
    }
}

// Moments of one pair (IN or CUT), T = accumulation type of the local
// integrals.  Sample acceptance is always decided in double.
// S = S0, S1[4], S2 upper triangle (00,01,02,03,11,12,13,22,23,33).
template <typename T>
__device__ inline void pair_moments(const double* X, double vol, const double* p, double d2, int code, int N,
                                    uint32_t key0, uint32_t key1, uint32_t q, uint32_t m, double* S) {
    if (code == C_IN) {
        double w = vol * 0.25;
        double s[15];
        for (int i = 0; i < 15; ++i) s[i] = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s[0] += w;
#pragma unroll
            for (int j = 0; j < 4; ++j) s[1 + j] += w * rule_w(r, j);
            int k = 5;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = i; j < 4; ++j) s[k++] += (w * rule_w(r, i)) * rule_w(r, j);
        }
        for (int i = 0; i < 15; ++i) S[i] = s[i];
        return;
    }
    double r2[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        double dx = X[3 * l] - p[0], dy = X[3 * l + 1] - p[1], dz = X[3 * l + 2] - p[2];
        r2[l] = (dx * dx + dy * dy) + dz * dz;
    }
    Mom<T> M;
#pragma unroll
    for (int i = 0; i < 15; ++i) M.s[i] = (T)0;
    CutGeom g;
    cut_setup<T>(X, p, d2, r2, vol, g, M);
    // relative vertex coordinates e_l = X_l - p
    double e0x = X[0] - p[0], e0y = X[1] - p[1], e0z = X[2] - p[2];
    double e1x = X[3] - p[0], e1y = X[4] - p[1], e1z = X[5] - p[2];
    double e2x = X[6] - p[0], e2y = X[7] - p[1], e2z = X[8] - p[2];
    double e3x = X[9] - p[0], e3y = X[10] - p[1], e3z = X[11] - p[2];
    // Monte Carlo sums: count, sum lambda_j (j = 1..3), sum lambda_i lambda_j (1 <= i <= j <= 3);
    // the lambda_0 terms follow from sum_l lambda_l = 1.
    T cnt = 0, a1 = 0, a2 = 0, a3 = 0, b11 = 0, b12 = 0, b13 = 0, b22 = 0, b23 = 0, b33 = 0;
    const double sc = 1.0 / 2097152.0;
    for (int s = 0; s < N; s += 2) {
        uint32_t w[4];
        philox4x32_10(q, m, (uint32_t)(s >> 1), 0u, key0, key1, w);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (s + h < N) {
                uint32_t L[4];
                lambda_u(w, h, L);
                double l0 = (double)L[0] * sc, l1 = (double)L[1] * sc, l2 = (double)L[2] * sc, l3 = (double)L[3] * sc;
                double dx = fma(l3, e3x, fma(l2, e2x, fma(l1, e1x, l0 * e0x)));
                double dy = fma(l3, e3y, fma(l2, e2y, fma(l1, e1y, l0 * e0y)));
                double dz = fma(l3, e3z, fma(l2, e2z, fma(l1, e1z, l0 * e0z)));
                double rr = fma(dz, dz, fma(dy, dy, dx * dx));
                double h0 = fma(g.c0[3], l3, fma(g.c0[2], l2, fma(g.c0[1], l1, g.c0[0] * l0)));
                double h1 = fma(g.c1[3], l3, fma(g.c1[2], l2, fma(g.c1[1], l1, g.c1[0] * l0)));
                bool inU = (h0 >= 0.0) && (h1 >= 0.0);
                bool acc = (rr < d2) && !inU;
                T x1 = acc ? (T)l1 : (T)0, x2 = acc ? (T)l2 : (T)0, x3 = acc ? (T)l3 : (T)0;
                cnt += acc ? (T)1 : (T)0;
                a1 += x1; a2 += x2; a3 += x3;
                b11 = fma(x1, (T)l1, b11); b12 = fma(x1, (T)l2, b12); b13 = fma(x1, (T)l3, b13);
                b22 = fma(x2, (T)l2, b22); b23 = fma(x2, (T)l3, b23); b33 = fma(x3, (T)l3, b33);
            }
        }
    }
    // complete the sums with the lambda_0 terms (exact in double for N <= 2048)
    double dc = (double)cnt, d1 = (double)a1, d2s = (double)a2, d3 = (double)a3;
    double c11 = (double)b11, c12 = (double)b12, c13 = (double)b13, c22 = (double)b22, c23 = (double)b23,
           c33 = (double)b33;
    double d0 = ((dc - d1) - d2s) - d3;
    double c01 = ((d1 - c11) - c12) - c13;
    double c02 = ((d2s - c12) - c22) - c23;
    double c03 = ((d3 - c13) - c23) - c33;
    double c00 = ((d0 - c01) - c02) - c03;
    double mc[15] = {dc, d0, d1, d2s, d3, c00, c01, c02, c03, c11, c12, c13, c22, c23, c33};
    double scale = vol / (double)N;
#pragma unroll
    for (int i = 0; i < 15; ++i) S[i] = (double)M.s[i] + scale * mc[i];
}

}  // namespace nlfem
