/*
 * TEST INFRASTRUCTURE ONLY -- part of the FP64 CPU oracle for the CTMRG step.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load it.
 * It shares no code with the GPU library.
 *
 * Cyclic two-sided Jacobi eigensolver for a real symmetric matrix, in plain C
 * with OpenMP.  This stands in for the diagonalization of the extended corner
 * matrix (Sec. III, Algorithm 3, the EigenExa call); the paper names no
 * algorithm for that step, so the oracle uses the textbook method whose
 * correctness is easiest to check: repeated plane rotations that zero one
 * off-diagonal pair at a time until the matrix is diagonal.
 *
 * Ordering: the round-robin ("chess tournament") ordering, in which every
 * round pairs all indices into n/2 disjoint pairs.  Disjoint rotations commute,
 * so all rotation angles of a round are computed from the matrix at the start
 * of the round and then applied together: first to the pairs of rows, then to
 * the pairs of columns.  Each sweep visits every pair (p,q) exactly once.
 *
 * Stopping rule: a pair is rotated only if |a_pq| > eps * sqrt(|a_pp a_qq|)
 * (the relative criterion of Demmel and Veselic); the iteration ends after a
 * sweep in which no pair was rotated.
 *
 * Layout: row-major, A[i*n + j].  Eigenvector j is column j of `evecs`
 * (evecs[i*n + j] is its component i).  Eigenvalues are returned unsorted.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int p, q;
    double c, s;
    int active;
} rot_t;

/* Rotation angle that zeroes a_pq (Golub & Van Loan, the symmetric 2x2 Schur
 * decomposition): with J = [[c, s], [-s, c]] acting on (p,q), J^T A J has a
 * zero in position (p,q). */
static void jacobi_angle(double app, double aqq, double apq, double *c, double *s, double *t_out)
{
    double tau = (aqq - app) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) {
        t = 0.5 / tau;
    } else {
        double sg = tau >= 0.0 ? 1.0 : -1.0;
        t = sg / (fabs(tau) + sqrt(1.0 + tau * tau));
    }
    *c = 1.0 / sqrt(1.0 + t * t);
    *s = t * (*c);
    *t_out = t;
}

/* Returns the number of sweeps used, or -1 if max_sweeps was reached. */
int oracle_jacobi(int n, double *A, double *evals, double *evecs, int max_sweeps)
{
    const double eps = 2.220446049250313e-16;
    if (n <= 0) return 0;
    memset(evecs, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) evecs[(size_t)i * n + i] = 1.0;
    if (n == 1) {
        evals[0] = A[0];
        return 0;
    }
    const int np = n + (n & 1); /* even number of players; index n is a dummy when n is odd */
    const int half = np / 2;
    rot_t *rot = (rot_t *)malloc(sizeof(rot_t) * half);
    double *newdiag = (double *)malloc(sizeof(double) * 2 * half);
    int sweeps = -1;

    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        long rotations = 0;
        for (int r = 0; r < np - 1; ++r) {
            /* Pairs of round r: (np-1, r) and ((r+i) mod (np-1), (r-i) mod (np-1)) for i=1..half-1. */
            for (int i = 0; i < half; ++i) {
                int p, q;
                if (i == 0) {
                    p = np - 1;
                    q = r;
                } else {
                    p = (r + i) % (np - 1);
                    q = (r - i + (np - 1)) % (np - 1);
                }
                if (p > q) { int tmp = p; p = q; q = tmp; }
                rot[i].p = p;
                rot[i].q = q;
                rot[i].active = 0;
                rot[i].c = 1.0;
                rot[i].s = 0.0;
                if (q >= n) continue; /* dummy partner */
                double apq = A[(size_t)p * n + q];
                double app = A[(size_t)p * n + p];
                double aqq = A[(size_t)q * n + q];
                if (apq == 0.0) continue;
                if (fabs(apq) <= eps * sqrt(fabs(app)) * sqrt(fabs(aqq))) continue;
                double c, s, t;
                jacobi_angle(app, aqq, apq, &c, &s, &t);
                rot[i].c = c;
                rot[i].s = s;
                rot[i].active = 1;
                newdiag[2 * i] = app - t * apq;
                newdiag[2 * i + 1] = aqq + t * apq;
                ++rotations;
            }
            /* Rows: A <- J^T A (pairs of rows p,q). */
#pragma omp parallel for schedule(static) if (n >= 128)
            for (int i = 0; i < half; ++i) {
                if (!rot[i].active) continue;
                double *rp = A + (size_t)rot[i].p * n;
                double *rq = A + (size_t)rot[i].q * n;
                const double c = rot[i].c, s = rot[i].s;
                for (int k = 0; k < n; ++k) {
                    double x = rp[k], y = rq[k];
                    rp[k] = c * x - s * y;
                    rq[k] = s * x + c * y;
                }
            }
            /* Columns: A <- A J, and the eigenvector matrix V <- V J. */
#pragma omp parallel for schedule(static) if (n >= 128)
            for (int k = 0; k < n; ++k) {
                double *ak = A + (size_t)k * n;
                double *vk = evecs + (size_t)k * n;
                for (int i = 0; i < half; ++i) {
                    if (!rot[i].active) continue;
                    const int p = rot[i].p, q = rot[i].q;
                    const double c = rot[i].c, s = rot[i].s;
                    double x = ak[p], y = ak[q];
                    ak[p] = c * x - s * y;
                    ak[q] = s * x + c * y;
                    x = vk[p];
                    y = vk[q];
                    vk[p] = c * x - s * y;
                    vk[q] = s * x + c * y;
                }
            }
            /* The 2x2 blocks take their exact rotated values. */
            for (int i = 0; i < half; ++i) {
                if (!rot[i].active) continue;
                const int p = rot[i].p, q = rot[i].q;
                A[(size_t)p * n + q] = 0.0;
                A[(size_t)q * n + p] = 0.0;
                A[(size_t)p * n + p] = newdiag[2 * i];
                A[(size_t)q * n + q] = newdiag[2 * i + 1];
            }
        }
        if (rotations == 0) {
            sweeps = sweep + 1;
            break;
        }
    }
    for (int i = 0; i < n; ++i) evals[i] = A[(size_t)i * n + i];
    free(rot);
    free(newdiag);
    return sweeps;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
