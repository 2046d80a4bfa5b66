/* Driver for the oracle's C part built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure, host only).
 *   argv: nx ny nz dx dy dz P m.bin cells.bin K octant_out.bin h_out.bin
 * Evaluates the real-space tensor octant and the direct demag sum at K target
 * cells for the magnetisation in m.bin (nx*ny*nz*3 doubles, Ms = 1), and
 * writes both as raw doubles. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_tensor_octant(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz, double P,
                          double *out);
void oracle_demag_direct_at(int64_t nx, int64_t ny, int64_t nz, const double *octant, const double *m,
                            const double *Ms, double Ms_scalar, int64_t K, const int64_t *tgt, double *out);

static void *slurp(const char *path, size_t bytes)
{
    FILE *f = fopen(path, "rb");
    if (!f) { perror(path); exit(2); }
    void *b = malloc(bytes);
    if (!b || fread(b, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return b;
}

static void spill(const char *path, const void *b, size_t bytes)
{
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(b, 1, bytes, f) != bytes) { perror(path); exit(2); }
    fclose(f);
}

int main(int argc, char **argv)
{
    if (argc != 13) { fprintf(stderr, "usage: nx ny nz dx dy dz P m cells K oct_out h_out\n"); return 2; }
    const int64_t nx = atoll(argv[1]), ny = atoll(argv[2]), nz = atoll(argv[3]);
    const double dx = atof(argv[4]), dy = atof(argv[5]), dz = atof(argv[6]), P = atof(argv[7]);
    const int64_t K = atoll(argv[10]);
    const size_t ncell = (size_t)(nx * ny * nz);
    double *m = slurp(argv[8], ncell * 3 * sizeof(double));
    int64_t *cells = slurp(argv[9], (size_t)K * 3 * sizeof(int64_t));
    double *oct = malloc(ncell * 6 * sizeof(double));
    double *h = malloc((size_t)K * 3 * sizeof(double));
    if (!oct || !h) return 2;
    oracle_tensor_octant(nx, ny, nz, dx, dy, dz, P, oct);
    oracle_demag_direct_at(nx, ny, nz, oct, m, NULL, 1.0, K, cells, h);
    spill(argv[11], oct, ncell * 6 * sizeof(double));
    spill(argv[12], h, (size_t)K * 3 * sizeof(double));
    free(m); free(cells); free(oct); free(h);
    return 0;
}
