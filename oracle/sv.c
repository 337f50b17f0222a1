/* O1 in plain C: the state vector psi = U_L ... U_1 e_0 in complex128.
 *
 * Part of the FP64 CPU oracle (test infrastructure only; never linked into
 * the library).  Same definition as statevector.py: qubit q is bit
 * (n-1-q) of the basis index; a one-qubit gate U mixes each pair of entries
 * whose indices differ only in that bit, new[b] = sum_c U[b][c] old[c]; T
 * multiplies the bit-1 entries by e^{i pi/4}; CZ negates entries whose two
 * bits are both 1.  The pair loop is split over OpenMP threads; every entry
 * is written by exactly one iteration, so the result does not depend on the
 * thread count.
 *
 * Gate kinds: 0 H, 1 sqrt X, 2 sqrt Y, 3 T, 4 CZ.  circuit is int32
 * [n_gates][4] = (kind, q0, q1, moment).  psi must hold 2^n doubles pairs
 * (re, im) and is overwritten.  Returns 0, or -1 for a bad gate.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

static void matrix_of(int kind, double complex u[2][2]) {
    const double r = 1.0 / sqrt(2.0);
    switch (kind) {
    case 0: u[0][0] = r; u[0][1] = r; u[1][0] = r; u[1][1] = -r; break;
    case 1:
        u[0][0] = 0.5 * (1 + I); u[0][1] = 0.5 * (1 - I);
        u[1][0] = 0.5 * (1 - I); u[1][1] = 0.5 * (1 + I); break;
    default: /* 2 */
        u[0][0] = 0.5 * (1 + I); u[0][1] = -0.5 * (1 + I);
        u[1][0] = 0.5 * (1 + I); u[1][1] = 0.5 * (1 + I); break;
    }
}

int oracle_statevector(int n, int n_gates, const int32_t *circuit, double *psi_out) {
    double complex *psi = (double complex *)psi_out;
    const int64_t dim = (int64_t)1 << n;
    memset(psi, 0, sizeof(double complex) * (size_t)dim);
    psi[0] = 1.0;
    const double complex tphase = cexp(I * M_PI / 4.0);
    for (int g = 0; g < n_gates; ++g) {
        const int kind = circuit[4 * g], q0 = circuit[4 * g + 1], q1 = circuit[4 * g + 2];
        if (q0 < 0 || q0 >= n) return -1;
        const int64_t m0 = (int64_t)1 << (n - 1 - q0);
        if (kind == 4) {
            if (q1 < 0 || q1 >= n || q1 == q0) return -1;
            const int64_t m1 = (int64_t)1 << (n - 1 - q1);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < dim; ++i)
                if ((i & m0) && (i & m1)) psi[i] = -psi[i];
        } else if (kind == 3) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < dim; ++i)
                if (i & m0) psi[i] *= tphase;
        } else if (kind >= 0 && kind <= 2) {
            double complex u[2][2];
            matrix_of(kind, u);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < dim; ++i) {
                if (i & m0) continue;
                const double complex a = psi[i], b = psi[i | m0];
                psi[i] = u[0][0] * a + u[0][1] * b;
                psi[i | m0] = u[1][0] * a + u[1][1] * b;
            }
        } else {
            return -1;
        }
    }
    return 0;
}
