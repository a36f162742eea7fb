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

// True if a face plane of the tet separates p from it by more than sqrt(lim):
// the distance from p to that plane bounds its distance to the closed tet
// from below.  Only used to skip the exact test for tets that are surely apart.
__device__ inline bool separated(const double* X, const double* p, double lim) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        // face opposite vertex f: (A, B, C) = the other three, D = vertex f
        const double* A = X + 3 * (f == 0 ? 1 : 0);
        const double* B = X + 3 * (f <= 1 ? 2 : 1);
        const double* C = X + 3 * (f <= 2 ? 3 : 2);
        const double* D = X + 3 * f;
        const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        const double sp = n[0] * (p[0] - A[0]) + n[1] * (p[1] - A[1]) + n[2] * (p[2] - A[2]);
        const double sd = n[0] * (D[0] - A[0]) + n[1] * (D[1] - A[1]) + n[2] * (D[2] - A[2]);
        if (sp * sd < 0.0 && sp * sp > lim * (n[0] * n[0] + n[1] * n[1] + n[2] * n[2])) return true;
    }
    return false;
}

// Classification against the open ball: 4 vertices inside -> IN, 1..3 ->
// CUT(n_in), none -> CUT(0) if the tet still meets the ball, else OUT.
// A bounding-box distance test and a separating-face-plane test first discard
// tets that are surely apart (margin 1e-9 relative, far above rounding), which
// leaves the result equal to the exact test.
// Fast part of the classification: the class, or -1 when only the exact
// closed-tet test can decide between CUT(0) and OUT.
__device__ inline int classify_fast(const double* X, const double* p, double d2) {
    int nin = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        double dx = X[3 * l] - p[0], dy = X[3 * l + 1] - p[1], dz = X[3 * l + 2] - p[2];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        nin += (r2 < d2) ? 1 : 0;
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
    return -1;
}

// Barycenter ((X0 + X1) + (X2 + X3)) / 4 in the open ball (strategy
// barycenter, Sec. 4.1).
__device__ inline bool barycenter_inside(const double* X, const double* p, double d2) {
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double c = ((X[i] + X[3 + i]) + (X[6 + i] + X[9 + i])) * 0.25;
        const double d = c - p[i];
        r2 = (i == 0) ? d * d : r2 + d * d;
    }
    return r2 < d2;
}

// Exact part for a tet with no vertex inside the open ball.
__device__ inline int classify_exact(const double* X, const double* p, double d2) {
    if (separated(X, p, d2 * (1.0 + 1e-9))) return C_OUT;
    return meets_ball(X, p, d2) ? C_CUT0 : C_OUT;
}

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
    if (separated(X, p, d2 * (1.0 + 1e-9))) return C_OUT;
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
        // three-input XORs as one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
        uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
}

// Philox counter of the sample pair j = floor(s / 2) (the paper leaves the
// sampling open, Sec. 4.2.2): pair keying (KEY 0) draws N samples of their
// own for every (outer point q, element m) pair, counter (q, m, j, 0);
// element keying (KEY 1) draws N samples per element, counter (m, j, 0, 1),
// the same points of E_m for every outer point.
template <int KEY>
__device__ __forceinline__ void mc_philox(uint32_t q, uint32_t m, uint32_t j, uint32_t k0, uint32_t k1, uint32_t* w) {
    if constexpr (KEY == 0) philox4x32_10(q, m, j, 0u, k0, k1, w);
    else philox4x32_10(m, j, 0u, 1u, k0, k1, w);
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
    // sorted as lo <= mid <= hi (the median as one v_med3_u32)
    const uint32_t lo = min(min(u0, u1), u2);
    const uint32_t hi = max(max(u0, u1), u2);
    const uint32_t mid = max(min(u0, u1), min(max(u0, u1), u2));
    L[0] = lo;
    L[1] = mid - lo;
    L[2] = hi - mid;
    L[3] = 2097152u - hi;
}

// A sample of the per-plan element-keyed table as one 64-bit word:
// L_1 | L_2 << 21 | L_3 << 42 (L_1, L_2 < 2^21, L_3 <= 2^21; L_0 follows from
// their sum 2^21).
__device__ __forceinline__ unsigned long long pack_lambda(const uint32_t* L) {
    return (unsigned long long)L[1] | ((unsigned long long)L[2] << 21) | ((unsigned long long)L[3] << 42);
}
__device__ __forceinline__ void unpack_lambda(uint32_t lo, uint32_t hi, uint32_t* L) {
    L[1] = lo & 0x1FFFFFu;
    L[2] = __builtin_amdgcn_alignbit(hi, lo, 21) & 0x1FFFFFu;
    L[3] = hi >> 10;
}

// ---------------------------------------------------------------------------
// Cut-pair geometry in the inner tet's barycentric space.  Everything below
// indexes its local arrays with compile-time constants only (runtime vertex
// ids pick values by selects or address global memory), so it stays in
// registers.
struct CutGeom {
    int nin;
    int nplanes;
    double c0[4], c1[4];  // U_I = E n {c0.l >= 0} [n {c1.l >= 0}]
};

// Hull point of U_I: the barycentric point (1 - t) e_a + t e_b, or the
// vertex e_a when b < 0.
struct HullPt {
    int a, b;
    double t;
};

// The cap region E_m minus U_I, sampled instead of the whole E_m when the
// caps are sampled on it.  It is star-shaped from the first outside vertex o
// (o lies outside every plane of U_I, and a point of E_m outside U_I lies
// outside one of them), so the cones from o over its faces that do not
// contain o tile it: one corner tet for n_in = 3, three tets for n_in = 1, 2
// (built in cut_build); n = 0 for CUT(0), which samples the whole element.
// Sub-tet j is (o, v[j][0], v[j][1], v[j][2]).
struct CornerGeom {
    int n, o;
    HullPt v[3][3];
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


__device__ __forceinline__ void hull_dense(const HullPt& h, double* e) {
#pragma unroll
    for (int l = 0; l < 4; ++l)
        e[l] = (h.b < 0) ? ((l == h.a) ? 1.0 : 0.0) : ((l == h.a) ? 1.0 - h.t : ((l == h.b) ? h.t : 0.0));
}

// functional vanishing on the barycentric points Q1, Q2, Q3, oriented
// non-negative on the inside vertices (bits of `inside`, summed in ascending
// vertex order)
__device__ inline void plane_dense(const double* Q1, const double* Q2, const double* Q3, unsigned inside, double* c) {
    c[0] = det3m(Q1[1], Q1[2], Q1[3], Q2[1], Q2[2], Q2[3], Q3[1], Q3[2], Q3[3]);
    c[1] = -det3m(Q1[0], Q1[2], Q1[3], Q2[0], Q2[2], Q2[3], Q3[0], Q3[2], Q3[3]);
    c[2] = det3m(Q1[0], Q1[1], Q1[3], Q2[0], Q2[1], Q2[3], Q3[0], Q3[1], Q3[3]);
    c[3] = -det3m(Q1[0], Q1[1], Q1[2], Q2[0], Q2[1], Q2[2], Q3[0], Q3[1], Q3[2]);
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
        if ((inside >> l) & 1u) s = s + c[l];
    if (s < 0.0)
#pragma unroll
        for (int l = 0; l < 4; ++l) c[l] = -c[l];
}

// sphere crossing on edge a (inside) -> b (outside); Xg = the inner tet's
// vertex coordinates ([4][3], global memory), r2a = |X_a - p|^2
__device__ __forceinline__ double edge_t(const double* Xg, const double* p, double d2, double r2a, int a, int b) {
    double ea[3] = {Xg[3 * a] - p[0], Xg[3 * a + 1] - p[1], Xg[3 * a + 2] - p[2]};
    double dv[3] = {Xg[3 * b] - Xg[3 * a], Xg[3 * b + 1] - Xg[3 * a + 1], Xg[3 * b + 2] - Xg[3 * a + 2]};
    double A = dot3(dv, dv);
    double B = dot3(ea, dv);
    double C = r2a - d2;
    double s = sqrt(B * B - A * C);
    // the stable root form picked by the sign of B, with a single division
    const bool neg = B <= 0.0;
    double t = (neg ? (s - B) : (-C)) / (neg ? A : (B + s));
    return t > 1.0 ? 1.0 : t;
}

// Moments of a subtet with barycentric vertex rows v0..v3 and volume V:
//   S0 = V, S1 = V/4 sum_a v_a, S2 = V/20 (sum_a v_a v_a^T + s s^T), s = sum_a v_a.
// These are the integrals of the affine barycentric coordinates over the
// subtet; the 4-point rule of Sec. 4.2.1 is exact for them (degree <= 2), so
// it gives the same values.  ti_moments (below) sums them over T_I in T.

// position of the n-th set bit of m (n = 0: lowest), -1 if there is none
__device__ __forceinline__ int nth_bit(unsigned m, int n) {
    for (int i = 0; i < n; ++i) m &= m - 1u;
    return __ffs(m) - 1;
}

// Build U_I = conv(I u P) (fullcaps construction), add the moments of its
// subdivision T_I to M, and set the half-space form of U_I used by the
// sample test.  With I and O the inside / outside vertices in ascending
// order and P_xy the sphere crossing on edge x -> y, the hull points are
//   n_in = 1: h0 = I0, h1 = P_I0O0, h2 = P_I0O1, h5 = P_I0O2 (h3 = h4 = I0);
//             T_I = the corner tet {0,1,2,5}; plane through (1,2,5)
//   n_in = 3: h0..h2 = I0..I2, h3 = P_I0O0, h4 = P_I1O0, h5 = P_I2O0;
//             T_I = {0,1,2,5}, {0,1,4,5}, {0,3,4,5}; plane through (3,4,5)
//   n_in = 2: h0 = I0, h1 = P_I0O0, h2 = P_I0O1, h3 = I1, h4 = P_I1O0, h5 = P_I1O1;
//             the quad (1,2,4,5) is split along the diagonal that gives the
//             larger (convex) volume, ties to the first:
//             T_I = {0,1,2,5}, {0,1,4,5}, {0,3,4,5}, planes (1,2,5), (1,4,5), or
//             T_I = {0,1,2,4}, {0,2,4,5}, {0,3,4,5}, planes (1,2,4), (2,4,5).
// Every lane runs the same instruction stream: the three subtets are always
// evaluated (zero-volume ones for n_in = 1 and n_in = 0), the hull points and
// planes are picked by selects.  sub(ti) receives T_I once (TISet).
struct TISet {
    const double *H0, *H1, *H2, *H3, *H4, *H5;  // dense barycentric rows of the hull points
    const double *XA, *YB;                      // alt ? H4 : H5 and alt ? H2 : H1
    bool alt;
    double Va, Vb, Vc;  // volumes of (H0, H1, H2, XA), (H0, YB, H4, H5), (H0, H3, H4, H5)
    // subtet s = 0, 1, 2 as four rows and its volume
    template <typename F>
    __device__ __forceinline__ void each(F&& f) const {
        f(H0, H1, H2, XA, Va);
        f(H0, YB, H4, H5, Vb);
        f(H0, H3, H4, H5, Vc);
    }
};

template <typename Sub>
__device__ __forceinline__ void cut_build(const double* Xg, const double* p, double d2, const double* r2, double vol,
                                          CutGeom& g, CornerGeom* cr, Sub&& sub) {
    unsigned in = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
        if (r2[l] < d2) in |= 1u << l;
    const unsigned out = (~in) & 15u;
    const int ni = __popc(in);
    const int I0 = nth_bit(in, 0), I1 = nth_bit(in, 1), I2 = nth_bit(in, 2);
    const int O0 = nth_bit(out, 0), O1 = nth_bit(out, 1), O2 = nth_bit(out, 2);
    auto r2of = [&](int a) { return a == 0 ? r2[0] : (a == 1 ? r2[1] : (a == 2 ? r2[2] : r2[3])); };
    // sphere crossings; an edge a lane does not use is replaced by (0, 1) and
    // its result is never selected
    auto cross = [&](bool used, int a, int b) {
        const int aa = used ? a : 0, bb = used ? b : 1;
        return HullPt{aa, bb, edge_t(Xg, p, d2, r2of(aa), aa, bb)};
    };
    const bool c1 = ni == 1, c2 = ni == 2, c3 = ni == 3, any = ni > 0;
    const HullPt x1 = cross(any, I0, O0);                          // P_I0O0
    const HullPt x2 = cross(any, c3 ? I1 : I0, c3 ? O0 : O1);      // P_I0O1 | P_I1O0 (n_in = 3)
    const HullPt x3 = cross(any, c1 ? I0 : (c2 ? I1 : I2), c1 ? O2 : (c2 ? O1 : O0));  // h5
    const HullPt x4 = cross(c2, I1, O0);                           // P_I1O0 (n_in = 2)
    const int v0 = any ? I0 : 0;
    const HullPt h0{v0, -1, 0.0};
    // (n_in = 0 lanes take h0 everywhere: their dummy crossings may be NaN)
    const HullPt h1 = c3 ? HullPt{I1, -1, 0.0} : (any ? x1 : h0);
    const HullPt h2 = c3 ? HullPt{I2, -1, 0.0} : (any ? x2 : h0);
    const HullPt h3 = c3 ? x1 : HullPt{c2 ? I1 : v0, -1, 0.0};
    const HullPt h4 = c3 ? x2 : (c2 ? x4 : h0);
    const HullPt h5 = any ? x3 : h0;
    // dense barycentric rows of the six hull points, built once
    double H0[4], H1[4], H2[4], H3[4], H4[4], H5[4];
    hull_dense(h0, H0);
    hull_dense(h1, H1);
    hull_dense(h2, H2);
    hull_dense(h3, H3);
    hull_dense(h4, H4);
    hull_dense(h5, H5);
    const double d125 = fabs(det3_bary(H0, H1, H2, H5)), d145 = fabs(det3_bary(H0, H1, H4, H5));
    const double d345 = fabs(det3_bary(H0, H3, H4, H5));
    const double d124 = fabs(det3_bary(H0, H1, H2, H4)), d245 = fabs(det3_bary(H0, H2, H4, H5));
    const double v1 = (d125 + d145) + d345, v2 = (d124 + d245) + d345;
    const bool alt = c2 && !(v1 >= v2);  // second diagonal
    if (cr) {
        // cones from o = O0 (P_xy: the crossing on edge x -> y):
        //   n_in = 3: (o; P_I0o, P_I1o, P_I2o)
        //   n_in = 1 (a = I0, c = O1, d = O2): (o; P_ao, P_ac, P_ad), (o; c, d, P_ad), (o; c, P_ad, P_ac)
        //   n_in = 2 (a = I0, b = I1, d = O1): (o; d, P_ad, P_bd), then the two triangles of
        //   U_I's inner quad on its diagonal: P_ao-P_bd: (o; P_ao, P_ad, P_bd), (o; P_ao, P_bo, P_bd);
        //   P_ad-P_bo (alt): (o; P_ao, P_ad, P_bo), (o; P_ad, P_bo, P_bd)
        const HullPt vc{O1, -1, 0.0}, vd{O2, -1, 0.0};
        cr->o = O0;
        cr->n = c3 ? 1 : ((c1 || c2) ? 3 : 0);
        auto set = [&](int j, const HullPt& a, const HullPt& b, const HullPt& c) {
            cr->v[j][0] = a; cr->v[j][1] = b; cr->v[j][2] = c;
        };
        set(0, c2 ? vc : x1, x2, x3);
        set(1, c1 ? vc : x1, c1 ? vd : x2, c1 ? x3 : (alt ? x4 : x3));
        set(2, c1 ? vc : (alt ? x2 : x1), c1 ? x3 : x4, c1 ? x2 : x3);
    }
    // subtets of T_I: (h0, h1, h2, alt ? h4 : h5), (h0, alt ? h2 : h1, h4, h5), (h0, h3, h4, h5)
    double XA[4], YB[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        XA[l] = alt ? H4[l] : H5[l];
        YB[l] = alt ? H2[l] : H1[l];
    }
    sub(TISet{H0, H1, H2, H3, H4, H5, XA, YB, alt, vol * (alt ? d124 : d125), vol * (alt ? d245 : d145), vol * d345});
    g.nin = ni;
    g.nplanes = any ? (c2 ? 2 : 1) : 0;
    // planes: c0 through (h3, h4, h5) for n_in = 3, else (h1, h2, alt ? h4 : h5);
    // c1 (n_in = 2) through (alt ? h2 : h1, h4, h5)
    double PA[4], PB[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        PA[l] = c3 ? H3[l] : H1[l];
        PB[l] = c3 ? H4[l] : H2[l];
    }
    plane_dense(PA, PB, XA, in, g.c0);
    plane_dense(YB, H4, H5, in, g.c1);
    // sample test: a missing plane is replaced by one that holds everywhere
    // (c = (1,1,1,1): c.lambda = 1 >= 0), and for n_in = 0 by one that never holds.
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (!c2) g.c1[l] = 1.0;
        if (!any) g.c0[l] = -1.0;
    }
}

// Moments S = S0, S1[4], S2 upper triangle (00,01,02,03,11,12,13,22,23,33)
// of one pair, in three pieces that the integration kernel folds into its
// sums one at a time (so that only one piece's state is live at once):
//   in_moments   the 4-point rule on the whole inner tet (class IN);
//   cut_det      the fullcaps construction of U_I and the 4-point rule on its
//                subtets (deterministic part of a cut pair); fills g;
//   cut_mc       the Monte Carlo part over E_m minus U_I inside the ball.
// T = accumulation type of the local integrals.  Sample acceptance is always
// decided in double.
__device__ inline void in_moments(double vol, double* S) {
    double w = vol * 0.25;
    for (int i = 0; i < 15; ++i) S[i] = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        S[0] += w;
#pragma unroll
        for (int j = 0; j < 4; ++j) S[1 + j] += w * rule_w(r, j);
        int k = 5;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = i; j < 4; ++j) S[k++] += (w * rule_w(r, i)) * rule_w(r, j);
    }
}

// Moments of T_I added to D (S0, S1 per subtet) and G.
// S2 = sum_s V_s/20 (sum_{a in s} v_a v_a^T + s_s s_s^T) is regrouped by
// hull point: sum_h W_h h h^T + sum_s V_s/20 s_s s_s^T, W_h = the sum of
// V_s/20 over the subtets holding h (14 + 14 multiply-adds per hull point and
// per subtet instead of 100 per subtet).
template <typename T>
__device__ __forceinline__ void ti_moments(const TISet& ti, double* D, double* G) {
    T g2[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) g2[k] = (T)0;
    auto outer = [&](const double* h, double W) {  // g2 += (W/20) h h^T
        const T w = (T)(W * 0.05);
        T hw[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) hw[l] = w * (T)h[l];
        int k = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = i; j < 4; ++j) {
                g2[k] = fma(hw[i], (T)h[j], g2[k]);
                ++k;
            }
    };
    ti.each([&](const double* v0, const double* v1, const double* v2, const double* v3, double V) {
        T sv[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) sv[l] = (T)(((v0[l] + v1[l]) + v2[l]) + v3[l]);
        const T w4 = (T)(V * 0.25);
        D[0] += V;
#pragma unroll
        for (int j = 0; j < 4; ++j) D[1 + j] += (double)(w4 * sv[j]);
        double s[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) s[l] = (double)sv[l];
        outer(s, V);
    });
    const double a = ti.alt ? ti.Va : 0.0, b = ti.alt ? 0.0 : ti.Va;
    outer(ti.H0, (ti.Va + ti.Vb) + ti.Vc);
    outer(ti.H1, ti.Va + (ti.alt ? 0.0 : ti.Vb));
    outer(ti.H2, ti.Va + (ti.alt ? ti.Vb : 0.0));
    outer(ti.H3, ti.Vc);
    outer(ti.H4, (a + ti.Vb) + ti.Vc);
    outer(ti.H5, (b + ti.Vb) + ti.Vc);
#pragma unroll
    for (int k = 0; k < 10; ++k) G[k] += (double)g2[k];
}

// cut_build with the moments of T_I added to D and G
template <typename T>
__device__ inline void cut_setup(const double* Xg, const double* p, double d2, const double* r2, double vol,
                                 CutGeom& g, double* D, double* G, CornerGeom* cr = nullptr) {
    cut_build(Xg, p, d2, r2, vol, g, cr, [&](const TISet& ti) { ti_moments<T>(ti, D, G); });
}

template <typename T>
__device__ inline void cut_det(const double* X, double vol, const double* p, double d2, CutGeom& g, double* D,
                               double* G, CornerGeom* cr = nullptr) {
    // X: the inner tet's vertex coordinates [4][3] in global memory; S0, S1
    // of the subdivision go to D[0..4] (overwritten), S2 is added to G[0..9]
    double r2[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        double dx = X[3 * l] - p[0], dy = X[3 * l + 1] - p[1], dz = X[3 * l + 2] - p[2];
        r2[l] = (dx * dx + dy * dy) + dz * dz;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) D[i] = 0.0;
    cut_setup<T>(X, p, d2, r2, vol, g, D, G, cr);
}

// |y - p|^2 of a sample as a quadratic form in its barycentrics (l_1..l_3,
// with l_0 eliminated): with e = X_0 - p and F_l = (X_l - p) - (X_0 - p),
//   |y - p|^2 = c + sum_l l_l (b_l + A_ll l_l + sum_{j>l} A_lj l_j),
// c = e.e, b_l = 2 e.F_l, A_ll = F_l.F_l, A_lj = 2 F_l.F_j (each dot product
// an FMA chain over x, y, z), evaluated as three inner FMA chains and one
// outer chain: 9 FMAs per sample.
__device__ __forceinline__ double dot3f(double ax, double ay, double az, double bx, double by, double bz) {
    return fma(az, bz, fma(ay, by, ax * bx));
}
struct BallForm {
    double c, b1, b2, b3, a11, a12, a13, a22, a23, a33;
    BallForm() = default;
    __device__ __forceinline__ BallForm(double ex, double ey, double ez, double f1x, double f1y, double f1z, double f2x,
                                        double f2y, double f2z, double f3x, double f3y, double f3z) {
        c = dot3f(ex, ey, ez, ex, ey, ez);
        b1 = 2.0 * dot3f(ex, ey, ez, f1x, f1y, f1z);
        b2 = 2.0 * dot3f(ex, ey, ez, f2x, f2y, f2z);
        b3 = 2.0 * dot3f(ex, ey, ez, f3x, f3y, f3z);
        a11 = dot3f(f1x, f1y, f1z, f1x, f1y, f1z);
        a12 = 2.0 * dot3f(f1x, f1y, f1z, f2x, f2y, f2z);
        a13 = 2.0 * dot3f(f1x, f1y, f1z, f3x, f3y, f3z);
        a22 = dot3f(f2x, f2y, f2z, f2x, f2y, f2z);
        a23 = 2.0 * dot3f(f2x, f2y, f2z, f3x, f3y, f3z);
        a33 = dot3f(f3x, f3y, f3z, f3x, f3y, f3z);
    }
    __device__ __forceinline__ double eval(double l1, double l2, double l3) const {
        const double t1 = fma(a13, l3, fma(a12, l2, fma(a11, l1, b1)));
        const double t2 = fma(a23, l3, fma(a22, l2, b2));
        const double t3 = fma(a33, l3, b3);
        return fma(l3, t3, fma(l2, t2, fma(l1, t1, c)));
    }
};

// Monte Carlo sums of one block of samples of a pair, and its moments.
//
// The sample barycentrics are lambda = L * 2^-21 with integer L (spacings of
// 21-bit uniforms).  With lambda_0 = 1 - lambda_1 - lambda_2 - lambda_3
// substituted, |y - p|^2 is the quadratic form of BallForm in lambda_1..3 and
// a plane value c . lambda = c_0 + sum_{l=1..3} lambda_l (c_l - c_0) an FMA
// chain over l = 1, 2, 3.  The loop works with L itself: the differences are
// prescaled by 2^-21 (exact), so every product with L equals the lambda
// form's product exactly and all roundings are those of the lambda form.  The
// sums are scaled back at the end (exact powers of two).
//
// Sums over the accepted samples are integers: the count and sum L_j
// (j = 1..3) in 32 bits, sum L_i L_j (1 <= i <= j <= 3) in 64 bits (one
// multiply-add each), exact for N <= 2047.  The L_0 terms follow exactly from
// sum_l L_l = 2^21, in integers or, equally exactly, in double (every partial
// sum is a multiple of 2^-42 below 2^11).  Both precisions of the local
// integrals therefore get the same, exact Monte Carlo moments.
struct McSums {
    uint32_t icnt = 0, ia1 = 0, ia2 = 0, ia3 = 0;
    uint64_t B11 = 0, B12 = 0, B13 = 0, B22 = 0, B23 = 0, B33 = 0;
    // sample L in the frame (bf, planes pl: p?0 + sum_l L_l p?l >= 0 both means
    // in U_I, rejected); accepted iff inside the open ball and not in U_I
    __device__ __forceinline__ void add(const BallForm& bf, const double* pl, double d2, const uint32_t* L) {
        double l1 = (double)L[1], l2 = (double)L[2], l3 = (double)L[3];
        double rr = bf.eval(l1, l2, l3);
        double h0 = fma(l3, pl[3], fma(l2, pl[2], fma(l1, pl[1], pl[0])));
        double h1 = fma(l3, pl[7], fma(l2, pl[6], fma(l1, pl[5], pl[4])));
        bool inU = (h0 >= 0.0) && (h1 >= 0.0);
        bool acc = (rr < d2) && !inU;
        // the sums under the lane mask (a branch, not selects)
        if (acc) {
            const uint32_t x1 = L[1], x2 = L[2], x3 = L[3];
            icnt += 1u;
            ia1 += x1; ia2 += x2; ia3 += x3;
            B11 += (uint64_t)x1 * x1; B12 += (uint64_t)x1 * x2; B13 += (uint64_t)x1 * x3;
            B22 += (uint64_t)x2 * x2; B23 += (uint64_t)x2 * x3; B33 += (uint64_t)x3 * x3;
        }
    }
    // moments of the accepted samples' coordinates, times scale, to S[15]
    template <typename T>
    __device__ __forceinline__ void finish(double scale, double* S) const {
        constexpr bool kF32 = sizeof(T) == 4;
        const double u = 1.0 / 2097152.0;
        // L_0 terms in integers (used by the float form below)
        const uint64_t TT = 2097152ull;
        const uint64_t A1 = ia1, A2 = ia2, A3 = ia3;
        const uint64_t A0 = (uint64_t)icnt * TT - A1 - A2 - A3;
        const uint64_t B01 = A1 * TT - B11 - B12 - B13, B02 = A2 * TT - B12 - B22 - B23,
                       B03 = A3 * TT - B13 - B23 - B33;
        const uint64_t B00 = A0 * TT - B01 - B02 - B03;
        double cnt = (double)icnt, a0 = (double)A0, a1 = (double)A1, a2 = (double)A2, a3 = (double)A3;
        double b00 = (double)B00, b01 = (double)B01, b02 = (double)B02, b03 = (double)B03, b11 = (double)B11,
               b12 = (double)B12, b13 = (double)B13, b22 = (double)B22, b23 = (double)B23, b33 = (double)B33;
        const double u2 = u * u;
        double dc = (double)cnt, d1 = (double)a1 * u, d2s = (double)a2 * u, d3 = (double)a3 * u;
        double c11 = (double)b11 * u2, c12 = (double)b12 * u2, c13 = (double)b13 * u2, c22 = (double)b22 * u2,
               c23 = (double)b23 * u2, c33 = (double)b33 * u2;
        double d0, c00, c01, c02, c03;
        if (kF32) {
            d0 = (double)a0 * u;
            c00 = (double)b00 * u2;
            c01 = (double)b01 * u2;
            c02 = (double)b02 * u2;
            c03 = (double)b03 * u2;
        } else {
            d0 = ((dc - d1) - d2s) - d3;
            c01 = ((d1 - c11) - c12) - c13;
            c02 = ((d2s - c12) - c22) - c23;
            c03 = ((d3 - c13) - c23) - c33;
            c00 = ((d0 - c01) - c02) - c03;
        }
        S[0] = scale * dc; S[1] = scale * d0; S[2] = scale * d1; S[3] = scale * d2s; S[4] = scale * d3;
        S[5] = scale * c00; S[6] = scale * c01; S[7] = scale * c02; S[8] = scale * c03; S[9] = scale * c11;
        S[10] = scale * c12; S[11] = scale * c13; S[12] = scale * c22; S[13] = scale * c23; S[14] = scale * c33;
    }
};

// The whole element's sample frame: ball form and U_I's planes, prescaled
__device__ __forceinline__ BallForm whole_frame(const double* X, const double* p, const CutGeom& g, double* pl) {
    const double u = 1.0 / 2097152.0;
    const double e0x = X[0] - p[0], e0y = X[1] - p[1], e0z = X[2] - p[2];
    const double f1x = ((X[3] - p[0]) - e0x) * u, f1y = ((X[4] - p[1]) - e0y) * u, f1z = ((X[5] - p[2]) - e0z) * u;
    const double f2x = ((X[6] - p[0]) - e0x) * u, f2y = ((X[7] - p[1]) - e0y) * u, f2z = ((X[8] - p[2]) - e0z) * u;
    const double f3x = ((X[9] - p[0]) - e0x) * u, f3y = ((X[10] - p[1]) - e0y) * u,
                 f3z = ((X[11] - p[2]) - e0z) * u;
    pl[0] = g.c0[0]; pl[1] = (g.c0[1] - g.c0[0]) * u; pl[2] = (g.c0[2] - g.c0[0]) * u; pl[3] = (g.c0[3] - g.c0[0]) * u;
    pl[4] = g.c1[0]; pl[5] = (g.c1[1] - g.c1[0]) * u; pl[6] = (g.c1[2] - g.c1[0]) * u; pl[7] = (g.c1[3] - g.c1[0]) * u;
    return BallForm(e0x, e0y, e0z, f1x, f1y, f1z, f2x, f2y, f2z, f3x, f3y, f3z);
}

// Sub-tet j of the cap region: its ball form, and planes that never hold
// (no U_I test)
__device__ __forceinline__ BallForm region_frame(const double* X, const double* p, const CornerGeom* cr, int j,
                                                 double* pl) {
    const double u = 1.0 / 2097152.0;
    const double* Xo = X + 3 * cr->o;
    const double e0x = Xo[0] - p[0], e0y = Xo[1] - p[1], e0z = Xo[2] - p[2];
    // point - p: X_a - p for a vertex, (X_a - p) + t (X_b - X_a) as one FMA for a crossing
    double fy[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const HullPt h = cr->v[j][l];
        const double* Xa = X + 3 * h.a;
        const double* Xb = X + 3 * (h.b < 0 ? h.a : h.b);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double e0c = c == 0 ? e0x : (c == 1 ? e0y : e0z);
            const double ev = h.b < 0 ? Xa[c] - p[c] : fma(h.t, Xb[c] - Xa[c], Xa[c] - p[c]);
            fy[l][c] = (ev - e0c) * u;
        }
    }
    pl[0] = -1.0; pl[1] = 0.0; pl[2] = 0.0; pl[3] = 0.0;
    pl[4] = 1.0; pl[5] = 0.0; pl[6] = 0.0; pl[7] = 0.0;
    return BallForm(e0x, e0y, e0z, fy[0][0], fy[0][1], fy[0][2], fy[1][0], fy[1][1], fy[1][2], fy[2][0], fy[2][1],
                    fy[2][2]);
}

// Folds the sums of sub-tet j's block (n_s samples) into S: its volume (the
// corner tet's |E| (1 - t_0)(1 - t_1)(1 - t_2), a cone tet's |E| |det of its
// barycentric rows|), the moments of its coordinates mu at weight |T_j| / n_s,
// mapped to E_m's as lambda = A mu with A[v][r] = component v of point r:
// S1 += A M1, S2 += A M2 A^T (as A M2, then times A^T).
template <typename T>
__device__ inline void region_fold(const CornerGeom* cr, int j, double vol, int n_s, const McSums& acc, double* S) {
    double A[4][4];
    {
        double R0[4], R1[4], R2[4], R3[4];
        hull_dense(HullPt{cr->o, -1, 0.0}, R0);
        hull_dense(cr->v[j][0], R1);
        hull_dense(cr->v[j][1], R2);
        hull_dense(cr->v[j][2], R3);
        vol = cr->n == 1 ? vol * (((1.0 - cr->v[0][0].t) * (1.0 - cr->v[0][1].t)) * (1.0 - cr->v[0][2].t))
                         : vol * fabs(det3_bary(R0, R1, R2, R3));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            A[v][0] = R0[v]; A[v][1] = R1[v]; A[v][2] = R2[v]; A[v][3] = R3[v];
        }
    }
    double Sj[15];
    acc.finish<T>(vol / (double)n_s, Sj);
    double M2[4][4];
    int k = 5;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = i; r < 4; ++r) {
            M2[i][r] = Sj[k];
            M2[r][i] = Sj[k];
            ++k;
        }
    S[0] += Sj[0];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double acc1 = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc1 = fma(A[v][r], Sj[1 + r], acc1);
        S[1 + v] += acc1;
    }
    double AM[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) a = fma(A[v][i], M2[i][r], a);
            AM[v][r] = a;
        }
    k = 5;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int w = v; w < 4; ++w) {
            double a = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) a = fma(AM[v][r], A[w][r], a);
            S[k++] += a;
        }
}

// The Monte Carlo part of a cut pair, over samples 0 <= s < N (Philox
// counters of mc_philox<KEY>, two samples per call; the whole-element loop
// makes two independent calls per iteration, and the sums are exact integers,
// so the loop's shape does not change them): uniform on E_m, those in
// U_I rejected; or, with the cap region on (VR, cr->n > 0), sub-tet j of n
// takes the samples floor(j N / n) <= s < floor((j + 1) N / n), N_j of them
// (N >= 3), with weight |T_j| / N_j and no U_I test, and its moments in the
// sub-tet's coordinates mu map to E_m's as lambda = sum_r mu_r row(T_j, r).
// Every lane runs the same sample loop (lanes of other classes in the wave
// do not serialise it).
// (cr: the cap region, used with VR; trow: with element keying and no cap
// region, element m's row of the per-plan sample table, the same samples
// that mc_philox<1> gives, or nullptr to draw them)
template <typename T, bool VR = false, int KEY = 0>
__device__ inline void cut_mc(const double* X, double vol, const double* p, double d2, const CutGeom& g, int N,
                              uint32_t key0, uint32_t key1, uint32_t q, uint32_t m, double* S,
                              const CornerGeom* cr, const unsigned long long* trow = nullptr) {
    double pl[8];
    if constexpr (!VR && KEY == 1) {
        if (trow) {
            const BallForm bf = whole_frame(X, p, g, pl);
            McSums acc;
            // blocks of eight samples (64 bytes per lane), the next block in
            // flight while one is tested; the row holds one padding block
            // past its last sample, so the read-ahead needs no branch
            const uint4* r4 = (const uint4*)trow;
            uint4 c[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] = r4[i];
            for (int s = 0; s < N; s += 8) {
                uint4 nx[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) nx[i] = r4[(s >> 1) + 4 + i];
#pragma unroll
                for (int h = 0; h < 8; ++h) {
                    if (s + h < N) {
                        const uint4 v = c[h >> 1];
                        uint32_t L[4];
                        if (h & 1) unpack_lambda(v.z, v.w, L);
                        else unpack_lambda(v.x, v.y, L);
                        acc.add(bf, pl, d2, L);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) c[i] = nx[i];
            }
            acc.finish<T>(vol / (double)N, S);
            return;
        }
    }
    if constexpr (!VR) {
        const BallForm bf = whole_frame(X, p, g, pl);
        McSums acc;
        for (int s = 0; s < N; s += 4) {
            uint32_t w[2][4];
            mc_philox<KEY>(q, m, (uint32_t)(s >> 1), key0, key1, w[0]);
            mc_philox<KEY>(q, m, (uint32_t)(s >> 1) + 1u, key0, key1, w[1]);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                if (s + h < N) {
                    uint32_t L[4];
                    lambda_u(w[h >> 1], h & 1, L);
                    acc.add(bf, pl, d2, L);
                }
            }
        }
        acc.finish<T>(vol / (double)N, S);
    } else {
        // nb = 0: the whole element (CUT(0)), 1: the corner tet, 3: three cone tets
        const int nb = cr->n;
#pragma unroll
        for (int i = 0; i < 15; ++i) S[i] = 0.0;
        BallForm bf;
        McSums acc;
        // the samples in three segments, the same for every lane of the wave
        // (N is): the cone tets' blocks.  A lane with one frame loads it before
        // the first segment and folds after the last; a lane with three loads
        // and folds one per segment.  (One site each keeps the kernel small.)
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            const int s0 = (j * N) / 3, s1 = ((j + 1) * N) / 3;
            if (j == 0 || nb == 3) bf = nb > 0 ? region_frame(X, p, cr, j, pl) : whole_frame(X, p, g, pl);
            for (int s = s0 & ~1; s < s1; s += 2) {
                uint32_t w[4];
                mc_philox<KEY>(q, m, (uint32_t)(s >> 1), key0, key1, w);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (s + h >= s0 && s + h < s1) {
                        uint32_t L[4];
                        lambda_u(w, h, L);
                        acc.add(bf, pl, d2, L);
                    }
                }
            }
            if (j == 2 || nb == 3) {
                const int n_s = nb == 3 ? s1 - s0 : N;
                if (nb > 0) {
                    region_fold<T>(cr, nb == 3 ? j : 0, vol, n_s, acc, S);
                } else {
                    acc.finish<T>(vol / (double)N, S);
                }
                acc = McSums();
            }
        }
    }
}

// whole-pair moments (the sum of the pieces), as the oracle reports them
template <typename T, bool VR = false, int KEY = 0>
__device__ inline void pair_moments(const double* X, double vol, const double* p, double d2, int code, int N,
                                    bool caps, uint32_t key0, uint32_t key1, uint32_t q, uint32_t m, double* S) {
    if (code == C_IN) {
        in_moments(vol, S);
        return;
    }
    CutGeom g;
    double D[5], G[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) G[i] = 0.0;
    CornerGeom cr;
    cut_det<T>(X, vol, p, d2, g, D, G, VR ? &cr : nullptr);
    if (caps) {
        cut_mc<T, VR, KEY>(X, vol, p, d2, g, N, key0, key1, q, m, S, &cr);
    } else {
#pragma unroll
        for (int i = 0; i < 15; ++i) S[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) S[i] = D[i] + S[i];
#pragma unroll
    for (int i = 0; i < 10; ++i) S[5 + i] = G[i] + S[5 + i];
}

// ---------------------------------------------------------------------------
// Paper-exact right-hand side (eq. Fh: g itself at the inner integration
// points).  g is a tensor polynomial
//   g(y) = sum_{a,b,c = 0..deg} coef[a + n1 (b + n1 c)] y1^a y2^b y3^c,  n1 = deg + 1,
// evaluated by Horner's rule along y3, then y2, then y1.
template <int DEG, typename CP>
__device__ __forceinline__ double gpoly_eval(CP coef, double y1, double y2, double y3) {
    constexpr int n1 = DEG + 1;
    double acc = 0.0;
#pragma unroll
    for (int a = DEG; a >= 0; --a) {
        double ay = 0.0;
#pragma unroll
        for (int b = DEG; b >= 0; --b) {
            double bz = 0.0;
#pragma unroll
            for (int c = DEG; c >= 0; --c) bz = bz * y3 + coef[a + n1 * (b + n1 * c)];
            ay = ay * y2 + bz;
        }
        acc = acc * y1 + ay;
    }
    return acc;
}

// e = g - g_h at the point with barycentrics lam in the inner tet X ([4][3]),
// g_h the affine interpolant of the nodal values gv of X's vertices
template <int DEG, typename CP>
__device__ __forceinline__ double g_defect_at(const double* X, const double* lam, const double* gv, CP coef) {
    double y[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = ((lam[0] * X[i] + lam[1] * X[3 + i]) + lam[2] * X[6 + i]) + lam[3] * X[9 + i];
    const double gh = ((lam[0] * gv[0] + lam[1] * gv[1]) + lam[2] * gv[2]) + lam[3] * gv[3];
    return gpoly_eval<DEG>(coef, y[0], y[1], y[2]) - gh;
}

// Integral of e = g - g_h over E_m n B_delta,h(p) with the inner rules of the
// pair: the 4-point rule of Sec. 4.2.1 on E_m (class IN) or on every subtet
// of T_I, and, when the caps are part of the pair, the accepted Monte Carlo
// samples of cut_mc (the same counters, the same acceptance test) with weight
// |E_m|/N each.  The matrix already carries the g_h part through the nodal
// constraint values, so this defect is what the right-hand side lacks.
template <int DEG, typename CP>
__device__ inline double pair_g_defect(const double* X, double vol, const double* p, double d2, int code, int N,
                                       bool caps, int keying, uint32_t key0, uint32_t key1, uint32_t q, uint32_t m,
                                       const double* gv, CP coef) {
    double acc = 0.0;
    if (code == C_IN) {
        const double w = vol * 0.25;
        for (int r = 0; r < 4; ++r) {
            double lam[4];
#pragma unroll
            for (int l = 0; l < 4; ++l) lam[l] = rule_w(r, l);
            acc += w * g_defect_at<DEG>(X, lam, gv, coef);
        }
        return acc;
    }
    double r2[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        double dx = X[3 * l] - p[0], dy = X[3 * l + 1] - p[1], dz = X[3 * l + 2] - p[2];
        r2[l] = (dx * dx + dy * dy) + dz * dz;
    }
    CutGeom g;
    cut_build(X, p, d2, r2, vol, g, nullptr, [&](const TISet& ti) {
        ti.each([&](const double* v0, const double* v1, const double* v2, const double* v3, double V) {
            const double w = V * 0.25;
            for (int r = 0; r < 4; ++r) {
                double lam[4];
#pragma unroll
                for (int l = 0; l < 4; ++l)
                    lam[l] = ((rule_w(r, 0) * v0[l] + rule_w(r, 1) * v1[l]) + rule_w(r, 2) * v2[l]) +
                             rule_w(r, 3) * v3[l];
                acc += w * g_defect_at<DEG>(X, lam, gv, coef);
            }
        });
    });
    if (!caps) return acc;
    // the counters and the acceptance test of cut_mc, term for term
    double sum = 0.0;
    auto take = [&](bool ok, const uint32_t* L) {
        if (ok) {
            const double u = 1.0 / 2097152.0;
            const double lam[4] = {(double)L[0] * u, (double)L[1] * u, (double)L[2] * u, (double)L[3] * u};
            sum += g_defect_at<DEG>(X, lam, gv, coef);
        }
    };
    {
        double pl[8];
        const BallForm bf = whole_frame(X, p, g, pl);
        for (int s = 0; s < N; s += 2) {
            uint32_t w[4];
            if (keying) mc_philox<1>(q, m, (uint32_t)(s >> 1), key0, key1, w);
            else mc_philox<0>(q, m, (uint32_t)(s >> 1), key0, key1, w);
            for (int h = 0; h < 2 && s + h < N; ++h) {
                uint32_t L[4];
                lambda_u(w, h, L);
                const double l1 = (double)L[1], l2 = (double)L[2], l3 = (double)L[3];
                const double rr = bf.eval(l1, l2, l3);
                const double h0 = fma(l3, pl[3], fma(l2, pl[2], fma(l1, pl[1], pl[0])));
                const double h1 = fma(l3, pl[7], fma(l2, pl[6], fma(l1, pl[5], pl[4])));
                take((rr < d2) && !((h0 >= 0.0) && (h1 >= 0.0)), L);
            }
        }
    }
    return acc + (vol / (double)N) * sum;
}

}  // namespace nlfem
