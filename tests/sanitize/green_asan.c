/* The oracle's C part (oracle/green.c) under AddressSanitizer and UBSan:
 * dense U and T matrices and streamed rows of a small sphere, checked for
 * finite entries and for rows that equal the dense (row-major) product. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_dense(int kind, int64_t nx, const double *X, int64_t ny, const double *Y,
                     const double *N, int same, double omega, double lam, double mu, double rho,
                     double self_re, double self_im, double complex *out);
int64_t oracle_matvec_rows(int kind, int64_t nx, const double *X, int64_t ny, const double *Y,
                           const double *N, int same, double omega, double lam, double mu,
                           double rho, double self_re, double self_im, int64_t nrows,
                           const int64_t *rows, int64_t nrhs, const double complex *b,
                           double complex *out);

int main(void) {
    const int n = 200;
    double *P = malloc(sizeof(double) * 3 * n);
    const double ga = M_PI * (3.0 - sqrt(5.0));
    for (int i = 0; i < n; ++i) {
        const double z = 1.0 - 2.0 * (i + 0.5) / n, r = sqrt(1.0 - z * z);
        P[3 * i] = r * cos(ga * i);
        P[3 * i + 1] = r * sin(ga * i);
        P[3 * i + 2] = z;
    }
    double complex *A = malloc(sizeof(double complex) * 9 * n * n);
    double complex *b = malloc(sizeof(double complex) * 3 * n);
    double complex *y = malloc(sizeof(double complex) * 3 * 8);
    int64_t rows[8] = {0, 1, 17, 63, 100, 150, 198, 199};
    for (int k = 0; k < 3 * n; ++k) b[k] = sin(0.7 * k) + I * cos(0.3 * k);
    for (int kind = 0; kind < 2; ++kind) {
        const int64_t bad = oracle_dense(kind, n, P, n, P, P, 1, 5.6, 2.0, 1.0, 1.0, 0.5, 0.0, A);
        if (bad) {
            printf("kind %d: %lld singular pairs\n", kind, (long long)bad);
            return 1;
        }
        for (int64_t k = 0; k < 9LL * n * n; ++k)
            if (!isfinite(creal(A[k])) || !isfinite(cimag(A[k]))) return 2;
        if (oracle_matvec_rows(kind, n, P, n, P, P, 1, 5.6, 2.0, 1.0, 1.0, 0.5, 0.0, 8, rows, 1, b, y))
            return 3;
        double err = 0, ref = 0;
        for (int q = 0; q < 8; ++q)
            for (int a = 0; a < 3; ++a) {
                double complex s = 0;
                for (int c = 0; c < 3 * n; ++c) s += A[(3 * rows[q] + a) * (int64_t)(3 * n) + c] * b[c];
                err += cabs(s - y[3 * q + a]);
                ref += cabs(s);
            }
        printf("kind %d: rows vs dense %.3e\n", kind, err / ref);
        if (!(err <= 1e-12 * ref)) return 4;
    }
    free(P); free(A); free(b); free(y);
    return 0;
}
