/*
 * Oracle (test infrastructure only; never linked into the HIP product path).
 *
 * The demagnetisation field at a few target cells as the plain O(N) sum over
 * every source cell of the convolution of eq. (4), with the sign made
 * explicit:  H_i = - sum_j N(r_i - r_j) M_j,  M_j = Ms_j m_j.
 *
 * N at a signed offset comes from the real-space octant N(|i|,|j|,|k|) by
 * the parity of each component: xx, yy, zz even in every axis; xy odd in x
 * and y; xz odd in x and z; yz odd in y and z.  Component order: xx, yy, zz,
 * xy, xz, yz.
 *
 * Sums over up to 2^34 source cells: every thread adds its share with
 * Neumaier's compensated summation and the thread partials are added the
 * same way, so the result carries a few units of rounding of the largest
 * terms, not of their count.  The numpy sum in field.demag_direct defines
 * the same quantity; the tests check the two against each other.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

typedef struct { double s, c; } ksum;

static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

static double kval(const ksum *k) { return k->s + k->c; }

/*
 * octant : (nx, ny, nz, 6) doubles, N at offsets 0 <= i < nx, ...
 * m      : (nx, ny, nz, 3) doubles
 * Ms     : (nx, ny, nz) doubles, or NULL for the scalar Ms_scalar
 * tgt    : (K, 3) int64 target cells
 * out    : (K, 3) doubles
 */
void oracle_demag_direct_at(int64_t nx, int64_t ny, int64_t nz, const double *octant, const double *m,
                            const double *Ms, double Ms_scalar, int64_t K, const int64_t *tgt, double *out)
{
    for (int64_t t = 0; t < K; ++t) {
        const int64_t ti = tgt[3 * t], tj = tgt[3 * t + 1], tk = tgt[3 * t + 2];
        ksum tot[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma omp parallel
        {
            ksum part[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma omp for schedule(static)
            for (int64_t I = 0; I < nx; ++I) {
                const int64_t di = ti - I, ai = di < 0 ? -di : di;
                const double sx = di < 0 ? -1.0 : 1.0;
                for (int64_t J = 0; J < ny; ++J) {
                    const int64_t dj = tj - J, aj = dj < 0 ? -dj : dj;
                    const double sy = dj < 0 ? -1.0 : 1.0;
                    for (int64_t Kz = 0; Kz < nz; ++Kz) {
                        const int64_t dk = tk - Kz, ak = dk < 0 ? -dk : dk;
                        const double sz = dk < 0 ? -1.0 : 1.0;
                        const int64_t src = (I * ny + J) * nz + Kz;
                        const double ms = Ms ? Ms[src] : Ms_scalar;
                        const double Mx = ms * m[3 * src], My = ms * m[3 * src + 1], Mz = ms * m[3 * src + 2];
                        const double *N = octant + ((ai * ny + aj) * nz + ak) * 6;
                        const double nxx = N[0], nyy = N[1], nzz = N[2];
                        const double nxy = N[3] * sx * sy, nxz = N[4] * sx * sz, nyz = N[5] * sy * sz;
                        kadd(&part[0], -(nxx * Mx + nxy * My + nxz * Mz));
                        kadd(&part[1], -(nxy * Mx + nyy * My + nyz * Mz));
                        kadd(&part[2], -(nxz * Mx + nyz * My + nzz * Mz));
                    }
                }
            }
#pragma omp critical
            {
                for (int a = 0; a < 3; ++a) {
                    kadd(&tot[a], part[a].s);
                    kadd(&tot[a], part[a].c);
                }
            }
        }
        for (int a = 0; a < 3; ++a) out[3 * t + a] = kval(&tot[a]);
    }
}
