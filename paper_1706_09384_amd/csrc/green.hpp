// Device evaluation of the 3x3 elastodynamic Green's tensors U and T.
//
// U = (1/mu)[G_ks I + ks^-2 Hess(G_ks - G_kp)] (eq. elasto_U rewritten with
// curl curl = grad div - Laplace), G_k = e^{ikr}/(4 pi r).  With d = x - y,
// r = |d|, dh = d/r, a = ks r, q = kp/ks:
//   U_ab = (A delta_ab + B dh_a dh_b) / (4 pi mu r)
//   A = e^{ia} + (E(a) - E(qa))/a^2,  B = (F(a) - F(qa))/a^2,
//   E(z) = e^{iz}(iz - 1),  F(z) = e^{iz}(3 - 3iz - z^2).
// T (traction in y of U with normal n(y), eq. elasto_T / Section 5.3):
//   T_ab = -[c1 n_a dh_b + c2((dh.n) delta_ab + dh_a n_b) + c3 (dh.n) dh_a dh_b]/(4 pi r^2)
//   c1 = (lambda/mu)(aA' - A + aB' + B) + 2B, c2 = aA' - A + B, c3 = 2(aB' - 3B).
// For small a the differences above cancel catastrophically (about
// 2 log10(1/a) digits), so below a threshold the Taylor series of the same
// functions is summed instead; every series term carries a factor (1 - q^m)
// and there is no cancellation.  Threshold / number of terms: 1.0 / 14 in
// float32, 0.5 / 17 in float64 (truncation below the type's rounding).
// The distance and the phases a, q a are formed in FP64 and reduced modulo
// 2 pi before the sine and cosine, so a float32 evaluation keeps its
// relative accuracy for large a (a float32 phase a = ks r would carry an
// absolute error of about 1e-7 a).
#pragma once

#include "common.hpp"

namespace hm {

template <typename R>
struct GreenParams {
    double ks_d, q_d;   // S wavenumber and kp / ks in FP64 (phases)
    R ks;        // S wavenumber
    R q;         // kp / ks
    R q2, q3;
    R lam_mu;    // lambda / mu
    R inv4pimu;  // 1 / (4 pi mu)
    R inv4pi;
    int kind;    // 0 = U, 1 = T
};

template <typename R>
struct SeriesCfg;
template <>
struct SeriesCfg<float> {
    static constexpr float below = 1.0f;
    static constexpr int last = 15;
};
template <>
struct SeriesCfg<double> {
    static constexpr double below = 0.5;
    static constexpr int last = 18;
};

__device__ inline void sincos_(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ inline void sincos_(double a, double *s, double *c) { sincos(a, s, c); }

// v - 2 pi k with k the nearest integer to v / (2 pi), in FP64.
__device__ inline double reduce_2pi(double v) {
    const double k = rint(v * 0.15915494309189535);
    return fma(-k, 6.283185307179586, v);
}

// Radial coefficient functions A, B, aA', aB' of the closed forms, given
// a, q a and the sines and cosines of both.
template <typename R>
__device__ inline void radial_coeffs(R a, R qa, R sa, R ca, R sq, R cq, const GreenParams<R> &g,
                                     cplx<R> &A, cplx<R> &B, cplx<R> &aAp, cplx<R> &aBp) {
    if (a < SeriesCfg<R>::below) {
        // t_m = i^m (1 - q^m) a^{m-2}/m!, summed with weights (m-1), (m-1)(m-3),
        // (m-1)(m-2), (m-1)(m-2)(m-3).
        R sAr = 0, sAi = 0, sBr = 0, sBi = 0, sPr = 0, sPi = 0, sQr = 0, sQi = 0;
        R qm = g.q2, am = 1, fact = 2;
#pragma unroll
        for (int m = 2; m <= SeriesCfg<R>::last; ++m) {
            const R c = (R(1) - qm) * am / fact;
            const R w1 = R(m - 1), w3 = R((m - 1) * (m - 3)), w2 = R((m - 1) * (m - 2)),
                    w4 = R((m - 1) * (m - 2) * (m - 3));
            switch (m & 3) {
                case 0: sAr += w1 * c; sBr += w3 * c; sPr += w2 * c; sQr += w4 * c; break;
                case 1: sAi += w1 * c; sBi += w3 * c; sPi += w2 * c; sQi += w4 * c; break;
                case 2: sAr -= w1 * c; sBr -= w3 * c; sPr -= w2 * c; sQr -= w4 * c; break;
                default: sAi -= w1 * c; sBi -= w3 * c; sPi -= w2 * c; sQi -= w4 * c; break;
            }
            qm *= g.q;
            am *= a;
            fact *= R(m + 1);
        }
        A = {ca + sAr, sa + sAi};
        B = {sBr, sBi};
        aAp = {-a * sa + sPr, a * ca + sPi};
        aBp = {sQr, sQi};
        return;
    }
    const R ia2 = R(1) / (a * a);
    // E(z) = e^{iz}(iz - 1)
    const R Ear = -ca - a * sa, Eai = a * ca - sa;
    const R Eqr = -cq - qa * sq, Eqi = qa * cq - sq;
    const R dEr = (Ear - Eqr) * ia2, dEi = (Eai - Eqi) * ia2;
    // F(z) = e^{iz}((3 - z^2) - 3iz)
    const R a2 = a * a, qa2 = qa * qa;
    const R Far = ca * (R(3) - a2) + R(3) * a * sa, Fai = sa * (R(3) - a2) - R(3) * a * ca;
    const R Fqr = cq * (R(3) - qa2) + R(3) * qa * sq, Fqi = sq * (R(3) - qa2) - R(3) * qa * cq;
    A = {ca + dEr, sa + dEi};
    B = {(Far - Fqr) * ia2, (Fai - Fqi) * ia2};
    // aA' = i a e^{ia} - e^{ia} + q^2 e^{iqa} - 2 dE
    aAp = {-a * sa - ca + g.q2 * cq - R(2) * dEr, a * ca - sa + g.q2 * sq - R(2) * dEi};
    // aB' = e^{ia}(1 - ia) - q^2 e^{iqa}(1 - iqa) - 2B
    aBp = {(ca + a * sa) - g.q2 * (cq + qa * sq) - R(2) * B.re,
           (sa - a * ca) - g.q2 * (sq - qa * cq) - R(2) * B.im};
}

// Direction dh = d / r, 1 / r and the radial coefficients at d = x - y.
template <typename R>
__device__ inline void radial_at(const GreenParams<R> &g, double dx, double dy, double dz, R (&d)[3],
                                 R &ir, cplx<R> &A, cplx<R> &B, cplx<R> &aAp, cplx<R> &aBp) {
    const double rd = sqrt(dx * dx + dy * dy + dz * dz);
    const double ird = 1.0 / rd;
    ir = R(ird);
    d[0] = R(dx * ird);
    d[1] = R(dy * ird);
    d[2] = R(dz * ird);
    const double ad = g.ks_d * rd, qad = g.q_d * ad;
    R sa, ca, sq, cq;
    if constexpr (sizeof(R) == 4) {
        sincos_(R(reduce_2pi(ad)), &sa, &ca);
        sincos_(R(reduce_2pi(qad)), &sq, &cq);
    } else {
        sincos_(R(ad), &sa, &ca);
        sincos_(R(qad), &sq, &cq);
    }
    radial_coeffs<R>(R(ad), R(qad), sa, ca, sq, cq, g, A, B, aAp, aBp);
}

// 3x3 block, row-major out[3a + b].  d = x - y (nonzero, FP64), n = unit
// normal at y.
template <typename R>
__device__ inline void green_block(const GreenParams<R> &g, double dx, double dy, double dz, R nx,
                                   R ny, R nz, cplx<R> out[9]) {
    R d[3], ir;
    cplx<R> A, B, aAp, aBp;
    radial_at<R>(g, dx, dy, dz, d, ir, A, B, aAp, aBp);
    if (g.kind == 0) {
        const R s = g.inv4pimu * ir;
        const cplx<R> sA = s * A, sB = s * B;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                const R dd = d[a] * d[b];
                cplx<R> v = dd * sB;
                if (a == b) v = v + sA;
                out[3 * a + b] = v;
                out[3 * b + a] = v;
            }
        return;
    }
    const R n[3] = {nx, ny, nz};
    const R dn = d[0] * nx + d[1] * ny + d[2] * nz;
    const cplx<R> c1 = g.lam_mu * (aAp - A + aBp + B) + R(2) * B;
    const cplx<R> c2 = aAp - A + B;
    const cplx<R> c3 = R(2) * (aBp - R(3) * B);
    const R s = -g.inv4pi * ir * ir;
    const cplx<R> s1 = s * c1, s2 = s * c2, s3 = (s * dn) * c3;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cplx<R> v = (n[a] * d[b]) * s1 + (d[a] * n[b]) * s2 + (d[a] * d[b]) * s3;
            if (a == b) v = v + dn * s2;
            out[3 * a + b] = v;
        }
}

template <typename R>
inline GreenParams<R> make_green_params(int kind, double omega, double lambda, double mu,
                                        double rho) {
    const double ks = omega * std::sqrt(rho / mu);
    const double kp = omega * std::sqrt(rho / (lambda + 2.0 * mu));
    const double q = ks > 0 ? kp / ks : std::sqrt(mu / (lambda + 2.0 * mu));
    GreenParams<R> g;
    g.ks_d = ks;
    g.q_d = q;
    g.ks = R(ks);
    g.q = R(q);
    g.q2 = R(q * q);
    g.q3 = R(q * q * q);
    g.lam_mu = R(lambda / mu);
    g.inv4pimu = R(1.0 / (4.0 * M_PI * mu));
    g.inv4pi = R(1.0 / (4.0 * M_PI));
    g.kind = kind;
    return g;
}

// P1 collocation operator (Section 4) on a triangle mesh whose vertices are
// both the collocation points and the column points.  All vertex numbers are
// cluster positions.
struct Colloc {
    const int32_t *tri;       // 3 vertices per element
    const int32_t *inc_ptr;   // elements around vertex j: inc[inc_ptr[j] .. inc_ptr[j + 1])
    const int32_t *inc;       // 4 e + k: element e, whose local vertex k is j
    const double *rule;       // (s, t, w) triples: nreg regular points, then nsing singular
    int32_t nreg, nsing;
};

// Cluster-ordered structure-of-arrays geometry in HBM.
struct Geometry {
    const double *x[3];   // row points
    const double *y[3];   // column points
    const double *n[3];   // normals at column points (T only)
    int same;
    Colloc mesh;          // mesh.tri == nullptr: point operator (eq. syst_a)
};

// Entry block (x_pi, vertex pj) of the collocation operator, row-major K[3a + b]:
//   sum over the elements e around pj of  int_{E_e} U(x_pi, y) v_pj(y) dS(y),
// v_pj the hat function of pj.  Each element integral is a collapsed
// Gauss-Legendre product rule: y = y_c + s (y_{c+1} - y_c) + s t (y_{c+2} -
// y_{c+1}), dS = s |(y_{c+1} - y_c) x (y_{c+2} - y_{c+1})| ds dt, hat values
// 1 - s, s (1 - t), s t at y_c, y_{c+1}, y_{c+2}; the rule collapses onto
// x_pi (singular rule) when x_pi is a vertex of E_e, where the factor s cancels
// the 1/r of U, and onto the element's first vertex (regular rule) otherwise.
// U is symmetric: six sums are kept.
template <typename R>
__device__ inline void colloc_block(const Geometry &g, const GreenParams<R> &gp, int pi, int pj,
                                    cplx<R> (&K)[9]) {
    const Colloc &m = g.mesh;
    const double x0 = g.x[0][pi], x1 = g.x[1][pi], x2 = g.x[2][pi];
    cplx<R> S[6];   // xx, yy, zz, xy, xz, yz
#pragma unroll
    for (int u = 0; u < 6; ++u) S[u] = {R(0), R(0)};
    const int32_t q1 = m.inc_ptr[pj + 1];
    for (int32_t q = m.inc_ptr[pj]; q < q1; ++q) {
        const int32_t ek = m.inc[q];
        const int32_t e = ek >> 2, k = ek & 3;
        const int32_t v0 = m.tri[3 * e], v1 = m.tri[3 * e + 1], v2 = m.tri[3 * e + 2];
        const int c = v0 == pi ? 0 : v1 == pi ? 1 : v2 == pi ? 2 : -1;
        const bool sing = c >= 0;
        const int c0 = sing ? c : 0;
        const int32_t va = c0 == 0 ? v0 : c0 == 1 ? v1 : v2;
        const int32_t vb = c0 == 0 ? v1 : c0 == 1 ? v2 : v0;
        const int32_t vc = c0 == 0 ? v2 : c0 == 1 ? v0 : v1;
        const int rel = (k - c0 + 3) % 3;   // position of pj in (va, vb, vc)
        double a[3], e1[3], e2[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a[d] = g.y[d][va];
            e1[d] = g.y[d][vb] - a[d];
            e2[d] = g.y[d][vc] - g.y[d][vb];
        }
        const double cx = e1[1] * e2[2] - e1[2] * e2[1];
        const double cy = e1[2] * e2[0] - e1[0] * e2[2];
        const double cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double two_area = sqrt(cx * cx + cy * cy + cz * cz);
        const double *rl = m.rule + (sing ? 3 * m.nreg : 0);
        const int32_t nq = sing ? m.nsing : m.nreg;
        for (int32_t qq = 0; qq < nq; ++qq) {
            const double s = rl[3 * qq], t = rl[3 * qq + 1], w = rl[3 * qq + 2];
            const double st = s * t;
            const double hat = rel == 0 ? 1.0 - s : rel == 1 ? s - st : st;
            R d[3], ir;
            cplx<R> A, B, aAp, aBp;
            radial_at<R>(gp, x0 - (a[0] + s * e1[0] + st * e2[0]), x1 - (a[1] + s * e1[1] + st * e2[1]),
                         x2 - (a[2] + s * e1[2] + st * e2[2]), d, ir, A, B, aAp, aBp);
            const R sc = R(w * two_area * hat) * gp.inv4pimu * ir;
            const cplx<R> sA = sc * A, sB = sc * B;
            S[0] = S[0] + (d[0] * d[0]) * sB + sA;
            S[1] = S[1] + (d[1] * d[1]) * sB + sA;
            S[2] = S[2] + (d[2] * d[2]) * sB + sA;
            S[3] = S[3] + (d[0] * d[1]) * sB;
            S[4] = S[4] + (d[0] * d[2]) * sB;
            S[5] = S[5] + (d[1] * d[2]) * sB;
        }
    }
    K[0] = S[0];
    K[4] = S[1];
    K[8] = S[2];
    K[1] = K[3] = S[3];
    K[2] = K[6] = S[4];
    K[5] = K[7] = S[5];
}

}  // namespace hm
