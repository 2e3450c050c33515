// Host build of the library's per-pair device math (seg_math.hpp), so the
// closed forms and the hand-written adjoint can be compared with the oracle
// on a machine without a GPU.  Test infrastructure only.
#include <cmath>
#include <cstdint>

#include "../../paper_2602_05492_amd/csrc/seg_math.hpp"

namespace {
template <class T>
struct HostM {
    static T log(T x) { return std::log(x); }
    static T log1p(T x) { return std::log1p(x); }
    static T rcp(T x) { return T(1) / x; }
    static T rsqrt(T x) { return T(1) / std::sqrt(x); }
    static T sqrt(T x) { return std::sqrt(x); }
    static T atan2(T y, T x) { return std::atan2(y, x); }
};

template <class T>
bem::SegGeom<T> geom(const double* s)
{
    bem::SegGeom<T> g;
    const double vx = s[2] - s[0], vy = s[3] - s[1];
    const double L2 = vx * vx + vy * vy > 1e-24 ? vx * vx + vy * vy : 0.0;   // degenerate-segment rule
    g.ax = (T)s[0]; g.ay = (T)s[1]; g.bx = (T)s[2]; g.by = (T)s[3];
    g.vx = (T)vx; g.vy = (T)vy; g.L2 = (T)L2;
    g.kd = L2 > 0.0 ? (T)(1.0 / (4.0 * bem::kPi * L2)) : T(0);
    g.ks = L2 > 0.0 ? (T)(1.0 / (8.0 * bem::kPi * L2 * std::sqrt(L2))) : T(0);
    g.iL2 = L2 > 0.0 ? (T)(1.0 / L2) : T(0);
    return g;
}

template <class T>
void moments(const double* x, int64_t n, const double* seg, int64_t K, double eps, double* out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < K; ++k) {
            const auto g = geom<T>(seg + 4 * k);
            const auto m = bem::seg_moments<T, HostM<T>>(g, (T)x[2 * i], (T)x[2 * i + 1], (T)(eps * eps));
            double* o = out + 4 * (i * K + k);
            o[0] = m.da; o[1] = m.db; o[2] = m.sa; o[3] = m.sb;
        }
}

template <class T>
void adjoint(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w, double* grad,
             double* mom)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < K; ++k) {
            const auto g = geom<T>(seg + 4 * k);
            const double* c = w + 4 * (i * K + k);
            bem::Moments<T> m;
            const auto r = bem::seg_adjoint<T, HostM<T>>(g, (T)x[2 * i], (T)x[2 * i + 1], (T)(eps * eps), (T)c[0],
                                                         (T)c[1], (T)c[2], (T)c[3], &m);
            double* o = grad + 4 * (i * K + k);
            o[0] = r.ax; o[1] = r.ay; o[2] = r.bx; o[3] = r.by;
            double* q = mom + 4 * (i * K + k);
            q[0] = m.da; q[1] = m.db; q[2] = m.sa; q[3] = m.sb;
        }
}
// The same gradients through the gradient-matrix form (one matrix per pair, applied to the
// cotangents).
template <class T>
void adjoint_matrix(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w,
                    double* grad)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < K; ++k) {
            const auto g = geom<T>(seg + 4 * k);
            const double* c = w + 4 * (i * K + k);
            const T e2 = (T)(eps * eps);
            const auto p = bem::pair_forward<T, HostM<T>>(g, (T)x[2 * i], (T)x[2 * i + 1], e2);
            const auto G = bem::pair_grad_matrix(g, p, e2);
            const auto r = bem::grad_apply(G, (T)c[0], (T)c[1], (T)c[2], (T)c[3]);
            double* o = grad + 4 * (i * K + k);
            o[0] = r.ax; o[1] = r.ay; o[2] = r.bx; o[3] = r.by;
        }
}
}  // namespace

extern "C" {
void hm_adjoint_matrix_f64(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w,
                           double* grad)
{ adjoint_matrix<double>(x, n, seg, K, eps, w, grad); }
void hm_adjoint_matrix_f32(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w,
                           double* grad)
{ adjoint_matrix<float>(x, n, seg, K, eps, w, grad); }
void hm_moments_f64(const double* x, int64_t n, const double* seg, int64_t K, double eps, double* out)
{ moments<double>(x, n, seg, K, eps, out); }
void hm_moments_f32(const double* x, int64_t n, const double* seg, int64_t K, double eps, double* out)
{ moments<float>(x, n, seg, K, eps, out); }
void hm_adjoint_f64(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w, double* grad,
                    double* mom)
{ adjoint<double>(x, n, seg, K, eps, w, grad, mom); }
void hm_adjoint_f32(const double* x, int64_t n, const double* seg, int64_t K, double eps, const double* w, double* grad,
                    double* mom)
{ adjoint<float>(x, n, seg, K, eps, w, grad, mom); }
void hm_beta_f64(const double* x, int64_t n, const double* el, int64_t M, double* out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < M; ++j) {
            const double* e = el + 4 * j;
            out[i * M + j] = bem::element_beta<double, HostM<double>>(e[0], e[1], e[2] - e[0], e[3] - e[1], x[2 * i],
                                                                      x[2 * i + 1]);
        }
}
}
