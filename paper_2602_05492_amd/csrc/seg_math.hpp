// seg_math.hpp - per-pair closed forms of the handle term and its adjoint.
//
// A straight handle segment a->b, seen from a sample x, contributes to the
// handle term of Eq. handleterm (regularised kernels, r^2 -> r^2 + eps^2,
// Sec. 3.1.3)
//     Md_a wd(a) + Md_b wd(b) + Ms_a wc(a) + Ms_b wc(b)
// where M?_a / M?_b are the integrals of the double-layer (d) or single-layer
// (s) kernel against the two linear hat functions of the segment.  Written in
// d = a - x, e = b - x, v = b - a (L2 = |v|^2):
//     C  = d x v          (= h L, signed)       D0 = d.v     D1 = e.v = D0 + L2
//     P  = d.e            R0 = |d|^2 + eps^2    R1 = |e|^2 + eps^2
//     l0 = log R0         ell = log(R1/R0) = log1p((2 D0 + L2)/R0)
//     Q  = sqrt(C^2 + eps^2 L2)   (= q L)       Dl = atan2(Q, P + eps^2) in [0, pi]
//     Md_b = C/(4 pi L2) (ell - 2 D0 Dl/Q)      Md_a = C/(4 pi L2) (2 D1 Dl/Q - ell)
//     S0 = L2 l0 + D1 ell - 2 L2 + 2 Q Dl       S1 = (2 D0 + L2)(l0 - 1) + R1 ell
//     Ms_b = (2 D0 S0 - L2 S1) / (8 pi L2^1.5)  Ms_a = (L2 S1 - 2 D1 S0) / (8 pi L2^1.5)
// ell is formed from R1 - R0 = 2 D0 + L2 rather than as a difference of two
// logarithms: far from a short segment ell ~ L/|d| is tiny, and the difference
// of two rounded logs would carry an absolute error that the factor C/L2 ~ |d|/L
// then amplifies (float32 error growing like |d|/L).
// (the four moments of the two kernels over the segment; Q^2 + (P+eps^2)^2 =
// R0 R1 is used by the adjoint).  With eps = 0 and C = 0 the double layer
// takes its principal value 0; R = 0 (eps = 0, x on an end point) gives the
// limits u log u^2 -> 0.
//
// The adjoint returns, for cotangents (wa, wb, sa, sb) of the four moments,
// the gradient of  wa Md_a + wb Md_b + sa Ms_a + sb Ms_b  with respect to the
// end points a and b (the parametric differentiation of Sec. 3.2: the
// integration variable runs over a fixed interval, so only the integrand
// depends on the end points).  It needs eps > 0 or a sample off the segment
// line.
//
// Everything is a template over the arithmetic type T and a math policy M
// supplying log, log1p, rcp, rsqrt and atan2 for T (atan2 is only called with
// a non-negative first argument: Q >= 0, and the subtended angle of an outer
// element seen from inside the domain), so the same code runs on gfx950 and in
// host-side unit tests.
#pragma once

#ifndef BEM_HD
#define BEM_HD __host__ __device__
#endif

namespace bem {

template <class T>
struct Moments {
    T da, db, sa, sb;
};

template <class T>
struct Grad4 {
    T ax, ay, bx, by;
};

// Per-segment constants that do not depend on the sample.
template <class T>
struct SegGeom {
    T ax, ay, bx, by;   // end points
    T vx, vy;           // b - a
    T L2;               // |b - a|^2
    T kd;               // 1 / (4 pi L2)
    T ks;               // 1 / (8 pi L2^1.5)
    T iL2;              // 1 / L2 (0 for a degenerate segment)
};

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kInv2Pi = 0.159154943091895335768883763372514362;

// l0 = log R0 and ell = log(R1/R0) = log1p(dR/R0), with the limits of the
// end-point cases R0 = 0 or R1 = 0 (eps = 0 and x on an end point) when Guard.
template <class T, class M, bool Guard>
BEM_HD inline void log_pair(T R0, T R1, T dR, T& l0, T& ell)
{
    if (!Guard) {
        l0 = M::log(R0);
        ell = M::log1p(dR * M::rcp(R0));
        return;
    }
    l0 = R0 > T(0) ? M::log(R0) : T(0);
    if (R0 > T(0) && R1 > T(0)) ell = M::log1p(dR * M::rcp(R0));
    else if (R0 > T(0)) ell = -l0;
    else ell = R1 > T(0) ? M::log(R1) : T(0);
}

// Forward moments of one pair.  X, Y: sample; eps2 = eps^2.  Guard = false
// drops the end-point and on-line limits (valid when both R0, R1 > 0 and
// Q > 0, e.g. a pair with the sample away from the segment).
template <class T, class M, bool Guard = true>
BEM_HD inline Moments<T> seg_moments(const SegGeom<T>& g, T X, T Y, T eps2)
{
    const T dx = g.ax - X, dy = g.ay - Y;
    const T ex = g.bx - X, ey = g.by - Y;
    const T C = dx * g.vy - dy * g.vx;
    const T D0 = dx * g.vx + dy * g.vy;
    const T D1 = D0 + g.L2;
    const T P = dx * ex + dy * ey;
    const T R0 = dx * dx + dy * dy + eps2;
    const T R1 = ex * ex + ey * ey + eps2;
    const T dR = T(2) * D0 + g.L2;                     // R1 - R0
    T l0, ell;
    log_pair<T, M, Guard>(R0, R1, dR, l0, ell);
    const T Q2 = C * C + eps2 * g.L2;
    const T iQ = Q2 > T(0) ? M::rsqrt(Q2) : T(0);     // eps = 0 on the segment line: principal value 0
    const T Q = Q2 * iQ;
    const T Dl = M::atan2(Q, P + eps2);
    const T gq = Dl * iQ;
    const T kd = C * g.kd;
    Moments<T> m;
    m.db = kd * (ell - T(2) * D0 * gq);
    m.da = kd * (T(2) * D1 * gq - ell);
    const T S0 = g.L2 * l0 + D1 * ell - T(2) * g.L2 + T(2) * Q * Dl;
    const T S1 = dR * (l0 - T(1)) + R1 * ell;
    m.sb = g.ks * (T(2) * D0 * S0 - g.L2 * S1);
    m.sa = g.ks * (g.L2 * S1 - T(2) * D1 * S0);
    return m;
}

// Forward state of one pair kept for the reverse pass.
template <class T>
struct PairState {
    T dx, dy, ex, ey;          // d = a - x, e = b - x
    T C, D0, D1, dR, R0, R1;
    T l0, ell, Q, Pe, Dl, iQ, gq, kdC, S0, S1, iR0, iR1;
};

template <class T, class M, bool Guard = true>
BEM_HD inline PairState<T> pair_forward(const SegGeom<T>& g, T X, T Y, T eps2)
{
    PairState<T> p;
    p.dx = g.ax - X; p.dy = g.ay - Y;
    p.ex = g.bx - X; p.ey = g.by - Y;
    p.C = p.dx * g.vy - p.dy * g.vx;
    p.D0 = p.dx * g.vx + p.dy * g.vy;
    p.D1 = p.D0 + g.L2;
    const T P = p.dx * p.ex + p.dy * p.ey;
    p.R0 = p.dx * p.dx + p.dy * p.dy + eps2;
    p.R1 = p.ex * p.ex + p.ey * p.ey + eps2;
    p.dR = T(2) * p.D0 + g.L2;
    log_pair<T, M, Guard>(p.R0, p.R1, p.dR, p.l0, p.ell);
    const T Q2 = p.C * p.C + eps2 * g.L2;
    p.iQ = Q2 > T(0) ? M::rsqrt(Q2) : T(0);
    p.Q = Q2 * p.iQ;
    p.Pe = P + eps2;
    p.Dl = M::atan2(p.Q, p.Pe);
    p.gq = p.Dl * p.iQ;
    p.kdC = p.C * g.kd;
    p.S0 = g.L2 * p.l0 + p.D1 * p.ell - T(2) * g.L2 + T(2) * p.Q * p.Dl;
    p.S1 = p.dR * (p.l0 - T(1)) + p.R1 * p.ell;
    p.iR0 = (!Guard || p.R0 > T(0)) ? M::rcp(p.R0) : T(0);
    p.iR1 = (!Guard || p.R1 > T(0)) ? M::rcp(p.R1) : T(0);
    return p;
}

template <class T>
BEM_HD inline Moments<T> pair_moments(const SegGeom<T>& g, const PairState<T>& p)
{
    Moments<T> m;
    m.db = p.kdC * (p.ell - T(2) * p.D0 * p.gq);
    m.da = p.kdC * (T(2) * p.D1 * p.gq - p.ell);
    m.sb = g.ks * (T(2) * p.D0 * p.S0 - g.L2 * p.S1);
    m.sa = g.ks * (g.L2 * p.S1 - T(2) * p.D1 * p.S0);
    return m;
}

// Reverse pass: gradient of wa Md_a + wb Md_b + sa Ms_a + sb Ms_b w.r.t. (a, b),
// the partials of ell = log R1 - log R0 being 1/R1 and -1/R0.
template <class T>
BEM_HD inline Grad4<T> pair_backward(const SegGeom<T>& g, const PairState<T>& p, T eps2, T wa, T wb, T sa, T sb)
{
    const T iL2 = g.iL2;
    // double layer: F_d = (C kd0) Ad,  kd0 = 1/(4 pi L2)
    const T Ad = (wb - wa) * p.ell + T(2) * p.gq * (wa * p.D1 - wb * p.D0);
    // single layer: F_s = ks As,  ks = 1/(8 pi L2^1.5)
    const T As = T(2) * p.S0 * (sb * p.D0 - sa * p.D1) + g.L2 * p.S1 * (sa - sb);

    T bC = Ad * g.kd;
    T bL2 = -p.kdC * Ad * iL2 + g.ks * p.S1 * (sa - sb) - T(1.5) * g.ks * As * iL2;
    T bell = p.kdC * (wb - wa);
    const T bg = T(2) * p.kdC * (wa * p.D1 - wb * p.D0);
    T bD1 = T(2) * p.kdC * p.gq * wa - T(2) * g.ks * p.S0 * sa;
    T bD0 = -T(2) * p.kdC * p.gq * wb + T(2) * g.ks * p.S0 * sb;
    const T bS0 = T(2) * g.ks * (sb * p.D0 - sa * p.D1);
    const T bS1 = g.ks * g.L2 * (sa - sb);
    // S0 = L2 l0 + D1 ell - 2 L2 + 2 Q Dl
    bL2 += bS0 * (p.l0 - T(2));
    T bl0 = bS0 * g.L2;
    bD1 += bS0 * p.ell;
    bell += bS0 * p.D1;
    T bQ = T(2) * bS0 * p.Dl;
    T bDl = T(2) * bS0 * p.Q;
    // S1 = dR (l0 - 1) + R1 ell,  dR = 2 D0 + L2
    const T bdR = bS1 * (p.l0 - T(1));
    bl0 += bS1 * p.dR;
    T bR1 = bS1 * p.ell;
    bell += bS1 * p.R1;
    bD0 += T(2) * bdR;
    bL2 += bdR;
    // gq = Dl / Q
    bDl += bg * p.iQ;
    bQ -= bg * p.gq * p.iQ;
    // l0 = log R0, ell = log R1 - log R0
    const T bR0 = (bl0 - bell) * p.iR0;
    bR1 += bell * p.iR1;
    // Dl = atan2(Q, Pe):  dDl/dQ = Pe/(R0 R1), dDl/dP = -Q/(R0 R1)
    const T iRR = p.iR0 * p.iR1;
    bQ += bDl * p.Pe * iRR;
    const T bP = -bDl * p.Q * iRR;
    // Q = sqrt(C^2 + eps2 L2)
    const T bQ2 = T(0.5) * bQ * p.iQ;
    bC += T(2) * p.C * bQ2;
    bL2 += eps2 * bQ2;
    // back to the vectors d = a - x, e = b - x (C = d x e, D0 = d.e - d.d, D1 = e.e - e.d,
    // P = d.e, R0 = d.d + eps2, R1 = e.e + eps2, L2 = |e - d|^2)
    const T ce = bD0 - bD1 + bP;            // coefficient of e in grad_d and of d in grad_e
    const T cd = T(2) * (bR0 - bD0);        // coefficient of d in grad_d
    const T cf = T(2) * (bR1 + bD1);        // coefficient of e in grad_e
    Grad4<T> r;
    r.ax = bC * p.ey + ce * p.ex + cd * p.dx - T(2) * bL2 * g.vx;
    r.ay = -bC * p.ex + ce * p.ey + cd * p.dy - T(2) * bL2 * g.vy;
    r.bx = -bC * p.dy + ce * p.dx + cf * p.ex + T(2) * bL2 * g.vx;
    r.by = bC * p.dx + ce * p.dy + cf * p.ey + T(2) * bL2 * g.vy;
    return r;
}

// The reverse pass above is linear in the cotangents.  Where one pair takes several
// cotangent sets (the three colour channels of a Jacobian row share the pair but not the
// end densities), the 4 x 4 matrix of that linear map is formed once and each set costs
// 16 multiply-adds.  Its columns are taken in the basis (wa, wb - wa, sa, sa - sb), a
// constant and a linearly varying density per layer, so that nearly equal end densities
// cancel before the products rather than after them:
//     grad = G (wa, wb - wa, sa, sa - sb),   rows ax, ay, bx, by.
// Each column is pair_backward's chain evaluated for that unit cotangent with the terms that
// vanish for it dropped (L2 iL2 = 1 used where it cancels a factor).
template <class T>
struct GradMatrix {
    T g[4][4];
};

template <class T>
BEM_HD inline void grad_column(const SegGeom<T>& g, const PairState<T>& p, T bC, T bL2, T ce, T cd, T cf,
                               GradMatrix<T>& G, int k)
{
    const T tL = T(2) * bL2;
    G.g[0][k] = bC * p.ey + ce * p.ex + cd * p.dx - tL * g.vx;
    G.g[1][k] = -bC * p.ex + ce * p.ey + cd * p.dy - tL * g.vy;
    G.g[2][k] = -bC * p.dy + ce * p.dx + cf * p.ex + tL * g.vx;
    G.g[3][k] = bC * p.dx + ce * p.dy + cf * p.ey + tL * g.vy;
}

template <class T>
BEM_HD inline GradMatrix<T> pair_grad_matrix(const SegGeom<T>& g, const PairState<T>& p, T eps2)
{
    GradMatrix<T> G;
    const T iRR = p.iR0 * p.iR1;
    const T PeR = p.Pe * iRR;
    const T k1 = T(0.5) * p.iQ * p.iQ * (PeR - p.gq);    // bQ2 per unit bg
    const T k2 = p.iQ * (p.Dl + p.Q * PeR);              // bQ2 per unit bS0
    const T k3 = p.Q * p.iQ * iRR;                       // -bP per unit bg
    const T k4 = T(2) * p.Q * p.Q * iRR;                 // -bP per unit bS0
    const T C2 = T(2) * p.C;
    const T kg = T(2) * p.kdC * p.gq;
    {   // wa = wb = 1: Ad = 2 gq L2, bg = 2 kdC L2, bD1 = -bD0 = 2 kdC gq, bell = 0
        const T bg = T(2) * p.kdC * g.L2;
        const T bQ2 = k1 * bg;
        const T bC = g.kd * (T(2) * p.gq * g.L2) + C2 * bQ2;
        const T bL2 = -kg + eps2 * bQ2;
        const T ce = -T(2) * kg - k3 * bg;
        grad_column(g, p, bC, bL2, ce, T(2) * kg, T(2) * kg, G, 0);
    }
    {   // wb = 1: Ad = ell - 2 gq D0, bg = -2 kdC D0, bD0 = -2 kdC gq, bell = kdC
        const T Ad = p.ell - T(2) * p.gq * p.D0;
        const T bg = -T(2) * p.kdC * p.D0;
        const T bQ2 = k1 * bg;
        const T bC = g.kd * Ad + C2 * bQ2;
        const T bL2 = -p.kdC * g.iL2 * Ad + eps2 * bQ2;
        const T ce = -kg - k3 * bg;
        const T cd = T(2) * (kg - p.kdC * p.iR0);
        const T cf = T(2) * p.kdC * p.iR1;
        grad_column(g, p, bC, bL2, ce, cd, cf, G, 1);
    }
    const T hS = T(2) * g.ks * p.S0;
    {   // sa = sb = 1: bS0 = -2 ks L2, bS1 = 0, As = -2 S0 L2, bD1 = -2 ks S0 + bS0 ell, bD0 = 2 ks S0
        const T b0 = -T(2) * g.ks * g.L2;
        const T bQ2 = k2 * b0;
        const T bC = C2 * bQ2;
        const T bL2 = T(1.5) * hS + b0 * (p.l0 - T(2)) + eps2 * bQ2;
        const T bD1 = -hS + b0 * p.ell;
        const T ce = hS - bD1 - k4 * b0;
        const T cd = T(2) * (-b0 * p.D0 * p.iR0 - hS);
        const T cf = T(2) * (b0 * p.D1 * p.iR1 + bD1);
        grad_column(g, p, bC, bL2, ce, cd, cf, G, 2);
    }
    {   // sb = -1: bS0 = -2 ks D0, bS1 = ks L2, As = L2 S1 - 2 S0 D0, bD1 = bS0 ell,
        //          bD0 = -2 ks S0 + 2 bS1 (l0 - 1)
        const T b0 = -T(2) * g.ks * p.D0;
        const T b1 = g.ks * g.L2;
        const T As = g.L2 * p.S1 - T(2) * p.S0 * p.D0;
        const T bdR = b1 * (p.l0 - T(1));
        const T bQ2 = k2 * b0;
        const T bC = C2 * bQ2;
        const T bL2 = g.ks * p.S1 - T(1.5) * g.ks * As * g.iL2 + b0 * (p.l0 - T(2)) + bdR + eps2 * bQ2;
        const T bell = b0 * p.D1 + b1 * p.R1;
        const T bD1 = b0 * p.ell;
        const T bD0 = -hS + T(2) * bdR;
        const T bl0 = b0 * g.L2 + b1 * p.dR;
        const T bR1 = b1 * p.ell + bell * p.iR1;
        const T bR0 = (bl0 - bell) * p.iR0;
        const T ce = bD0 - bD1 - k4 * b0;
        grad_column(g, p, bC, bL2, ce, T(2) * (bR0 - bD0), T(2) * (bR1 + bD1), G, 3);
    }
    return G;
}

// grad = G (wa, wb - wa, sa, sa - sb)
template <class T>
BEM_HD inline Grad4<T> grad_apply(const GradMatrix<T>& G, T wa, T wb, T sa, T sb)
{
    const T u[4] = {wa, wb - wa, sa, sa - sb};
    T r[4];
    for (int i = 0; i < 4; ++i) r[i] = G.g[i][0] * u[0] + G.g[i][1] * u[1] + G.g[i][2] * u[2] + G.g[i][3] * u[3];
    return Grad4<T>{r[0], r[1], r[2], r[3]};
}

// Gradient of wa Md_a + wb Md_b + sa Ms_a + sb Ms_b w.r.t. (a, b), and the
// moments themselves in *mom when mom != nullptr.
template <class T, class M, bool Guard = true>
BEM_HD inline Grad4<T> seg_adjoint(const SegGeom<T>& g, T X, T Y, T eps2,
                                   T wa, T wb, T sa, T sb, Moments<T>* mom)
{
    const PairState<T> p = pair_forward<T, M, Guard>(g, X, Y, eps2);
    if (mom) *mom = pair_moments(g, p);
    return pair_backward(g, p, eps2, wa, wb, sa, sb);
}

// Double layer of a constant unit density over an outer element with the
// exact kernel: beta(x) = -int dG/dn_y dy = (signed angle subtended at x)/2pi.
template <class T, class M>
BEM_HD inline T element_beta(T ax, T ay, T vx, T vy, T X, T Y)
{
    const T dx = ax - X, dy = ay - Y;
    const T ex = dx + vx, ey = dy + vy;
    const T C = dx * vy - dy * vx;
    const T P = dx * ex + dy * ey;
    return M::atan2(C, P) * T(kInv2Pi);
}

// Cubic Bernstein weights at t.
template <class T>
BEM_HD inline void bernstein3(T t, T w[4])
{
    const T s = T(1) - t;
    w[0] = s * s * s;
    w[1] = T(3) * s * s * t;
    w[2] = T(3) * s * t * t;
    w[3] = t * t * t;
}

// Weights of the polyline vertex at t on the handle's geometry parameters: the four cubic
// Bernstein weights of the control points, or (1 - t, t, 0, 0) on the end points of a
// straight handle (model 1).
template <class T>
BEM_HD inline void vertex_weights(int model, T t, T w[4])
{
    if (model == 1) {
        w[0] = T(1) - t;
        w[1] = t;
        w[2] = w[3] = T(0);
    } else {
        bernstein3(t, w);
    }
}

}  // namespace bem
