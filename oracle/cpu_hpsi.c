/*
 * Oracle: FP64 H psi on the host CPU with OpenMP (TEST INFRASTRUCTURE ONLY).
 *
 * Used to time the CPU baseline next to the GPU.  It applies the same
 * operator as the Python oracle (Sec. 5): the 25-point finite-difference
 * kinetic stencil through a neighbour table, the local potential product and
 * the Kleinman-Bylander projectors of eq. (6) in two parts (projections, then
 * the sum of projector functions times stored integrals, one atom at a time).
 * States are stored block by block with the state index fastest (Sec. 4,
 * Fig. "memory_layout" (b)): psi[blk][point][B].
 *
 * Built with -ffp-contract=off so each product and sum is rounded as written.
 */
#include <stdint.h>
#include <string.h>

void oracle_hpsi_f64(int64_t np, int nblk, int B,
                     const int64_t *nbr,      /* [np][3][2][M], -1 = outside */
                     int M, const double *c,  /* c[0..M] */
                     double h, const double *vloc,
                     const double *psi, double *hpsi,
                     int nat, const int64_t *sph_ptr, const int64_t *sph_idx,
                     const double *gamma,     /* [nnz][4] */
                     const double *D,         /* [nat][4] */
                     double *proj)            /* scratch [nat][4][B] */
{
    const double pre = -0.5 / (h * h);
    const double dv = h * h * h;
    const int nn = 3 * 2 * M;
    for (int blk = 0; blk < nblk; ++blk) {
        const double *x = psi + (int64_t)blk * np * B;
        double *y = hpsi + (int64_t)blk * np * B;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < np; ++p) {
            double acc[64];
            const double *xp = x + p * B;
            for (int s = 0; s < B; ++s) acc[s] = 3.0 * c[0] * xp[s];
            const int64_t *nb = nbr + p * nn;
            for (int a = 0; a < 3; ++a)
                for (int sg = 0; sg < 2; ++sg)
                    for (int m = 1; m <= M; ++m) {
                        int64_t q = nb[(a * 2 + sg) * M + (m - 1)];
                        if (q < 0) continue;
                        const double *xq = x + q * B;
                        const double cm = c[m];
                        for (int s = 0; s < B; ++s) acc[s] = acc[s] + cm * xq[s];
                    }
            double *yp = y + p * B;
            const double v = vloc[p];
            for (int s = 0; s < B; ++s) yp[s] = pre * acc[s] + v * xp[s];
        }
        if (nat == 0) continue;
        /* part 1: projections */
#pragma omp parallel for schedule(dynamic)
        for (int A = 0; A < nat; ++A) {
            double sum[4][64];
            memset(sum, 0, sizeof(sum));
            for (int64_t e = sph_ptr[A]; e < sph_ptr[A + 1]; ++e) {
                const double *xq = x + sph_idx[e] * B;
                const double *ga = gamma + e * 4;
                for (int i = 0; i < 4; ++i)
                    for (int s = 0; s < B; ++s) sum[i][s] = sum[i][s] + ga[i] * xq[s];
            }
            for (int i = 0; i < 4; ++i)
                for (int s = 0; s < B; ++s)
                    proj[((int64_t)A * 4 + i) * B + s] = dv * sum[i][s] * D[A * 4 + i];
        }
        /* part 2: scatter, one atom at a time (points of one sphere are distinct) */
        for (int A = 0; A < nat; ++A) {
            const double *pa = proj + (int64_t)A * 4 * B;
#pragma omp parallel for schedule(static)
            for (int64_t e = sph_ptr[A]; e < sph_ptr[A + 1]; ++e) {
                double *yq = y + sph_idx[e] * B;
                const double *ga = gamma + e * 4;
                for (int s = 0; s < B; ++s) {
                    double t = ga[0] * pa[s];
                    t = t + ga[1] * pa[B + s];
                    t = t + ga[2] * pa[2 * B + s];
                    t = t + ga[3] * pa[3 * B + s];
                    yq[s] = yq[s] + t;
                }
            }
        }
    }
}

/* Threads the parallel loops above use (the OpenMP default team size). */
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
