/*
 * Plain FP64 CPU oracle for the elastodynamic Green's tensors.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, includes or calls
 * this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark load it.
 *
 * What it computes (paper, Section 1, eqs. (elasto_U) and (elasto_T), and the
 * component form of Section 5.3):
 *
 *   U(x,y) = (1/(rho w^2)) [ curl curl (G_ks I) - grad div (G_kp I) ],
 *   G_k(r) = e^{i k r} / (4 pi r),  k_s^2 = rho w^2 / mu, k_p^2 = rho w^2/(lambda+2mu).
 *
 * Using curl curl = grad div - Laplace and (Laplace + k^2) G_k = 0 away from
 * r = 0 this is U = (1/mu) [ G_ks I + k_s^-2 Hess(G_ks - G_kp) ].  With
 * d = x - y, r = |d|, dh = d/r, a = k_s r, q = k_p/k_s, E(z) = e^{iz}(iz-1),
 * F(z) = e^{iz}(3 - 3iz - z^2), the Hessian of e^{ikr}/r is
 * r^-3 [E(kr) delta + F(kr) dh dh^T], so
 *
 *   U_ab = (A delta_ab + B dh_a dh_b) / (4 pi mu r),
 *   A = e^{ia} + (E(a) - E(qa))/a^2,   B = (F(a) - F(qa))/a^2.
 *
 * T is the traction of each column of U taken in y with normal n(y)
 * (Section 5.3): T_ab = C_agts d/dy_s U_bt n_g with the isotropic elasticity
 * tensor C_agts = lambda d_ag d_ts + mu (d_at d_gs + d_as d_gt).  Carrying the
 * y-derivative through the radial form gives
 *
 *   T_ab = -[ c1 n_a dh_b + c2 ((dh.n) d_ab + dh_a n_b) + c3 (dh.n) dh_a dh_b ] / (4 pi r^2)
 *   c1 = (lambda/mu)(aA' - A + aB' + B) + 2B,  c2 = aA' - A + B,  c3 = 2 (aB' - 3B)
 *
 * where ' is d/da.  Below a = 0.5 the differences E(a) - E(qa), F(a) - F(qa)
 * cancel, so the Taylor series of the same functions is used instead:
 * with t_m = i^m (1 - q^m) a^{m-2} / m!,  m >= 2,
 *   A = e^{ia} + sum (m-1) t_m,          B = sum (m-1)(m-3) t_m,
 *   aA' = i a e^{ia} + sum (m-1)(m-2) t_m,  aB' = sum (m-1)(m-2)(m-3) t_m.
 *
 * The dense matrix of eq. (syst_a) has 3x3 block (i,j) = U(x_i, y_j) or
 * T(x_i, y_j) (normal at y_j), rows 3i+alpha, columns 3j+beta.  When the two
 * clouds are the same set, the diagonal blocks i = j (where the kernel is
 * singular) are replaced by s I3 with a caller-given complex s.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex zc;

#define ORACLE_SERIES_BELOW 0.5

static void radial_closed(double a, double q, zc *A, zc *B, zc *aAp, zc *aBp)
{
    const zc ea = cexp(I * a), eqa = cexp(I * q * a);
    const double qa = q * a, a2 = a * a;
    const zc Ea = ea * (I * a - 1.0), Eqa = eqa * (I * qa - 1.0);
    const zc Fa = ea * (3.0 - 3.0 * I * a - a2), Fqa = eqa * (3.0 - 3.0 * I * qa - qa * qa);
    const zc dE = (Ea - Eqa) / a2;
    *A = ea + dE;
    *B = (Fa - Fqa) / a2;
    *aAp = I * a * ea - ea + q * q * eqa - 2.0 * dE;
    *aBp = ea * (1.0 - I * a) - eqa * (q * q - I * q * q * q * a) - 2.0 * (*B);
}

static void radial_series(double a, double q, zc *A, zc *B, zc *aAp, zc *aBp)
{
    const zc ea = cexp(I * a);
    zc sA = 0, sB = 0, sAp = 0, sBp = 0;
    /* t_m = i^m (1 - q^m) a^(m-2) / m! built incrementally. */
    zc im = -1.0;            /* i^2 */
    double qm = q * q;       /* q^2 */
    double am = 1.0;         /* a^0 */
    double fact = 2.0;       /* 2! */
    for (int m = 2; m < 60; ++m) {
        const zc t = im * (1.0 - qm) * am / fact;
        const double m1 = m - 1.0, m2 = m - 2.0, m3 = m - 3.0;
        sA += m1 * t;
        sB += m1 * m3 * t;
        sAp += m1 * m2 * t;
        sBp += m1 * m2 * m3 * t;
        if (m > 6 && cabs(t) * (m1 * m2 * m3 + 1.0) < 1e-18 * (cabs(sA) + cabs(sB) + 1e-300))
            break;
        im *= I;
        qm *= q;
        am *= a;
        fact *= (m + 1.0);
    }
    *A = ea + sA;
    *B = sB;
    *aAp = I * a * ea + sAp;
    *aBp = sBp;
}

/* Radial coefficient functions; exported for the tests. out = {A, B, aA', aB'}. */
void oracle_radial(double a, double q, double complex *out)
{
    if (a < ORACLE_SERIES_BELOW)
        radial_series(a, q, &out[0], &out[1], &out[2], &out[3]);
    else
        radial_closed(a, q, &out[0], &out[1], &out[2], &out[3]);
}

void oracle_radial_branch(double a, double q, int series, double complex *out)
{
    if (series)
        radial_series(a, q, &out[0], &out[1], &out[2], &out[3]);
    else
        radial_closed(a, q, &out[0], &out[1], &out[2], &out[3]);
}

/*
 * One 3x3 block, row-major out[3*alpha + beta].
 * kind 0 = U, 1 = T (nrm = unit normal at y, ignored for U).
 * Returns 0 on success, 1 if x == y (the kernel is singular there).
 */
int oracle_green_block(int kind, const double *x, const double *y, const double *nrm,
                       double omega, double lambda, double mu, double rho, double complex *out)
{
    const double ks = omega * sqrt(rho / mu);
    const double kp = omega * sqrt(rho / (lambda + 2.0 * mu));
    const double q = (ks > 0.0) ? kp / ks : sqrt(mu / (lambda + 2.0 * mu));
    const double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r == 0.0) {
        for (int k = 0; k < 9; ++k) out[k] = NAN;
        return 1;
    }
    const double dh[3] = {d[0] / r, d[1] / r, d[2] / r};
    zc c[4];
    oracle_radial(ks * r, q, c);
    const zc A = c[0], B = c[1], aAp = c[2], aBp = c[3];
    if (kind == 0) {
        const double s = 1.0 / (4.0 * M_PI * mu * r);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                out[3 * a + b] = s * ((a == b ? A : 0.0) + B * (dh[a] * dh[b]));
        return 0;
    }
    const double dn = dh[0] * nrm[0] + dh[1] * nrm[1] + dh[2] * nrm[2];
    const zc c1 = (lambda / mu) * (aAp - A + aBp + B) + 2.0 * B;
    const zc c2 = aAp - A + B;
    const zc c3 = 2.0 * (aBp - 3.0 * B);
    const double s = -1.0 / (4.0 * M_PI * r * r);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            out[3 * a + b] = s * (c1 * nrm[a] * dh[b] + c2 * ((a == b ? dn : 0.0) + dh[a] * nrm[b]) +
                                  c3 * dn * dh[a] * dh[b]);
    return 0;
}

/* Block (i, j) of the system matrix, honouring the self-block rule. */
static int entry_block(int kind, const double *X, const double *Y, const double *N, int64_t i,
                       int64_t j, int same, double omega, double lambda, double mu, double rho,
                       zc self, zc *blk)
{
    if (same && i == j) {
        for (int k = 0; k < 9; ++k) blk[k] = 0.0;
        blk[0] = blk[4] = blk[8] = self;
        return 0;
    }
    return oracle_green_block(kind, X + 3 * i, Y + 3 * j, N ? N + 3 * j : NULL, omega, lambda,
                              mu, rho, blk);
}

/*
 * Dense matrix (3 nx) x (3 ny), row-major complex128.  Returns the number of
 * singular (coincident, non-self) pairs met.
 */
int64_t oracle_dense(int kind, int64_t nx, const double *X, int64_t ny, const double *Y,
                     const double *N, int same, double omega, double lambda, double mu, double rho,
                     double self_re, double self_im, double complex *out)
{
    const zc self = self_re + I * self_im;
    const int64_t ld = 3 * ny;
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : bad)
    for (int64_t i = 0; i < nx; ++i) {
        zc blk[9];
        for (int64_t j = 0; j < ny; ++j) {
            bad += entry_block(kind, X, Y, N, i, j, same, omega, lambda, mu, rho, self, blk);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    out[(3 * i + a) * ld + 3 * j + b] = blk[3 * a + b];
        }
    }
    return bad;
}

/*
 * Streamed dense product for selected row points, without storing the matrix:
 * out[(3k + a) * nrhs + c] = sum_j sum_b K_ab(x_rows[k], y_j) b[(3j + b) * nrhs + c].
 * b and out are row-major complex128 with nrhs columns.
 */
int64_t oracle_matvec_rows(int kind, int64_t nx, const double *X, int64_t ny, const double *Y,
                           const double *N, int same, double omega, double lambda, double mu,
                           double rho, double self_re, double self_im, int64_t nrows,
                           const int64_t *rows, int64_t nrhs, const double complex *b,
                           double complex *out)
{
    const zc self = self_re + I * self_im;
    int64_t bad = 0;
    (void)nx;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t i = rows[k];
        zc *o = out + 3 * k * nrhs;
        memset(o, 0, sizeof(zc) * 3 * nrhs);
        zc blk[9];
        for (int64_t j = 0; j < ny; ++j) {
            bad += entry_block(kind, X, Y, N, i, j, same, omega, lambda, mu, rho, self, blk);
            const zc *bj = b + 3 * j * nrhs;
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    const zc kab = blk[3 * a + bb];
                    for (int64_t c = 0; c < nrhs; ++c) o[a * nrhs + c] += kab * bj[bb * nrhs + c];
                }
        }
    }
    return bad;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
