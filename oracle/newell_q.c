/*
 * Oracle (test infrastructure only; never linked into the HIP product path).
 *
 * Demag tensor of two equal rectangular cells, as the cell-averaged dipolar
 * kernel N(r) of the demagnetisation convolution (paper, Implementation
 * section, eq. (4); the paper takes N from Newell's formulas, Newell,
 * Williams & Dunlop 1993).
 *
 *   near field (|r|_2 <= P * max(dx,dy,dz)):  Newell f / g auxiliary
 *       functions combined with the 27-point second-difference stencil,
 *       evaluated in IEEE binary128 (__float128) so that the binary64 result
 *       is correctly rounded in all but pathological cases;
 *   far field  (|r|_2 >  P * max(dx,dy,dz)):  27-point dipole quadrature whose
 *       nodes match the 2nd and 4th moments of the cell-pair displacement
 *       distribution (error O((d/r)^6)), evaluated in x87 extended precision.
 *
 * The paper prints neither formula; the reading is stated in the design notes.
 * Component order everywhere: xx, yy, zz, xy, xz, yz.
 */
#include <quadmath.h>
#include <math.h>
#include <stdint.h>

typedef __float128 qf;

/* An odd component vanishes on the plane where its odd axis offset is zero;
 * the stencil sums reach that zero only up to rounding, so set it exactly. */
static void zero_odd_planes(int64_t i, int64_t j, int64_t k, double *out)
{
    if (i == 0 || j == 0) out[3] = 0.0;
    if (i == 0 || k == 0) out[4] = 0.0;
    if (j == 0 || k == 0) out[5] = 0.0;
}


/* Newell f: even in every argument. */
static qf newell_f(qf x, qf y, qf z)
{
    x = fabsq(x); y = fabsq(y); z = fabsq(z);
    qf x2 = x * x, y2 = y * y, z2 = z * z;
    qf R = sqrtq(x2 + y2 + z2);
    qf r = 0, p;
    p = y * (z2 - x2) / 2;
    if (p != 0) r += p * asinhq(y / sqrtq(x2 + z2));
    p = z * (y2 - x2) / 2;
    if (p != 0) r += p * asinhq(z / sqrtq(x2 + y2));
    p = x * y * z;
    if (p != 0) r -= p * atanq(y * z / (x * R));
    r += (2 * x2 - y2 - z2) * R / 6;
    return r;
}

/* Newell g: odd in x, odd in y, even in z. */
static qf newell_g(qf x, qf y, qf z)
{
    qf s = ((x < 0) != (y < 0)) ? -1 : 1;
    if (x == 0 || y == 0) s = 0;   /* odd in x and y: vanishes on both planes */
    x = fabsq(x); y = fabsq(y); z = fabsq(z);
    qf x2 = x * x, y2 = y * y, z2 = z * z;
    qf R = sqrtq(x2 + y2 + z2);
    qf r = 0, p;
    p = x * y * z;
    if (p != 0) r += p * asinhq(z / sqrtq(x2 + y2));
    p = y * (3 * z2 - y2) / 6;
    if (p != 0) r += p * asinhq(x / sqrtq(y2 + z2));
    p = x * (3 * z2 - x2) / 6;
    if (p != 0) r += p * asinhq(y / sqrtq(x2 + z2));
    p = z * z2 / 6;
    if (p != 0) r -= p * atanq(x * y / (z * R));
    p = z * y2 / 2;
    if (p != 0) r -= p * atanq(x * z / (y * R));
    p = z * x2 / 2;
    if (p != 0) r -= p * atanq(y * z / (x * R));
    r -= x * y * R / 3;
    return s * r;
}

/* sum over e in {-1,0,1}^3 of w(e) fn(X+e1 a, Y+e2 b, Z+e3 c), w = prod(2 | -1);
 * also accumulates sum |w fn| into *scale (the cancellation scale). */
static qf stencil27(qf (*fn)(qf, qf, qf), qf X, qf Y, qf Z, qf a, qf b, qf c, qf *scale)
{
    qf acc = 0, sc = 0;
    for (int e1 = -1; e1 <= 1; ++e1)
        for (int e2 = -1; e2 <= 1; ++e2)
            for (int e3 = -1; e3 <= 1; ++e3) {
                qf w = (qf)((e1 == 0 ? 2 : -1) * (e2 == 0 ? 2 : -1) * (e3 == 0 ? 2 : -1));
                qf t = w * fn(X + e1 * a, Y + e2 * b, Z + e3 * c);
                acc += t;
                sc += fabsq(t);
            }
    *scale = sc;
    return acc;
}

/* Newell tensor at lattice offset (i,j,k) of cells (dx,dy,dz), binary128.
 * out[6] in xx,yy,zz,xy,xz,yz; scale[6] (nullable) = sum|w f| / (4 pi V). */
void oracle_newell(int64_t i, int64_t j, int64_t k, double dx, double dy, double dz,
                   double *out, double *scale)
{
    qf a = dx, b = dy, c = dz;
    qf X = (qf)i * a, Y = (qf)j * b, Z = (qf)k * c;
    qf norm = 1 / (4 * M_PIq * a * b * c);
    qf v[6], s[6];
    v[0] = stencil27(newell_f, X, Y, Z, a, b, c, &s[0]);   /* xx: f(x,y,z) */
    v[1] = stencil27(newell_f, Y, X, Z, b, a, c, &s[1]);   /* yy: f(y,x,z) */
    v[2] = stencil27(newell_f, Z, Y, X, c, b, a, &s[2]);   /* zz: f(z,y,x) */
    v[3] = stencil27(newell_g, X, Y, Z, a, b, c, &s[3]);   /* xy: g(x,y,z) */
    v[4] = stencil27(newell_g, X, Z, Y, a, c, b, &s[4]);   /* xz: g(x,z,y) */
    v[5] = stencil27(newell_g, Y, Z, X, b, c, a, &s[5]);   /* yz: g(y,z,x) */
    for (int q = 0; q < 6; ++q) {
        out[q] = (double)(v[q] * norm);
        if (scale) scale[q] = (double)(s[q] * norm);
    }
    zero_odd_planes(i, j, k, out);
}

/* Far-field rule: average of the point-dipole tensor over 27 displaced nodes
 * r + s (e1 dx, e2 dy, e3 dz), s = sqrt(2/5), weights prod(7/12 | 5/24). */
void oracle_far(int64_t i, int64_t j, int64_t k, double dx, double dy, double dz, double *out)
{
    typedef long double ld;
    const ld s = sqrtl(0.4L);
    const ld V = (ld)dx * dy * dz;
    ld acc[6] = {0, 0, 0, 0, 0, 0};
    for (int e1 = -1; e1 <= 1; ++e1)
        for (int e2 = -1; e2 <= 1; ++e2)
            for (int e3 = -1; e3 <= 1; ++e3) {
                ld w = (e1 == 0 ? 7.0L / 12 : 5.0L / 24) * (e2 == 0 ? 7.0L / 12 : 5.0L / 24) *
                       (e3 == 0 ? 7.0L / 12 : 5.0L / 24);
                ld x = ((ld)i + e1 * s) * dx, y = ((ld)j + e2 * s) * dy, z = ((ld)k + e3 * s) * dz;
                ld r2 = x * x + y * y + z * z;
                ld r5 = r2 * r2 * sqrtl(r2);
                ld q = w / r5;
                acc[0] += q * (r2 - 3 * x * x);
                acc[1] += q * (r2 - 3 * y * y);
                acc[2] += q * (r2 - 3 * z * z);
                acc[3] += q * (-3 * x * y);
                acc[4] += q * (-3 * x * z);
                acc[5] += q * (-3 * y * z);
            }
    const ld pref = V / (4 * 3.14159265358979323846264338327950288L);
    for (int q = 0; q < 6; ++q) out[q] = (double)(acc[q] * pref);
    zero_odd_planes(i, j, k, out);
}

/* The tensor definition: Newell inside the switch radius, the far rule outside.
 * P <= 0 means Newell everywhere. */
void oracle_tensor_at(int64_t i, int64_t j, int64_t k, double dx, double dy, double dz,
                      double P, double *out)
{
    double dmax = dx > dy ? dx : dy;
    if (dz > dmax) dmax = dz;
    long double x = (long double)i * dx, y = (long double)j * dy, z = (long double)k * dz;
    long double r2 = x * x + y * y + z * z, lim = (long double)P * dmax;
    if (P <= 0 || r2 <= lim * lim)
        oracle_newell(i, j, k, dx, dy, dz, out, 0);
    else
        oracle_far(i, j, k, dx, dy, dz, out);
}

/* Many offsets at once: ijk[3*n], out[6*n]. OpenMP-parallel. */
void oracle_tensor_many(int64_t n, const int64_t *ijk, double dx, double dy, double dz,
                        double P, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n; ++t)
        oracle_tensor_at(ijk[3 * t], ijk[3 * t + 1], ijk[3 * t + 2], dx, dy, dz, P, out + 6 * t);
}

/* The real-space octant N(i,j,k), 0<=i<nx, 0<=j<ny, 0<=k<nz, layout
 * [i][j][k][6]. */
void oracle_tensor_octant(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                          double P, double *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t k = 0; k < nz; ++k)
                oracle_tensor_at(i, j, k, dx, dy, dz, P, out + 6 * ((i * ny + j) * nz + k));
}
