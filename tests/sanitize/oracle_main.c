/* A small driver of the CPU oracle for the AddressSanitizer / UBSan build
 * (tests/test_sanitizers.py): a 2-level nest over a sloping coast with a
 * child straddling the shoreline (an L of two touching blocks: a mask leaves
 * out the north-east corner of its rectangle), the elliptic source, 300
 * steps, and the correctly rounded cube root over a range of depths and near
 * binade edges.  Exit 0 when every value stays finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny, parent, off_i, off_j;
    double dx, ox, oy;
    double *h, *eta, *M, *N, *zmax, *M2, *N2, *clip;
    const uint8_t *mask;
} ora_level;
typedef struct {
    int32_t nlev;
    int32_t bc[4];
    ora_level *lv;
    double dt, g, manning, eps;
    int64_t steps;
} ora_domain;

void ora_step(ora_domain *d, int64_t nsteps);
void ora_set_source(ora_domain *d, double xc, double yc, double a, double b, double theta, double amp, int shape);
double ora_cbrt_rn(double x);

static void alloc_level(ora_level *L, int nx, int ny)
{
    L->nx = nx;
    L->ny = ny;
    L->h = calloc((size_t)nx * ny, sizeof(double));
    L->eta = calloc((size_t)nx * ny, sizeof(double));
    L->zmax = calloc((size_t)nx * ny, sizeof(double));
    L->clip = calloc((size_t)nx * ny, sizeof(double));
    L->M = calloc((size_t)(nx + 1) * ny, sizeof(double));
    L->M2 = calloc((size_t)(nx + 1) * ny, sizeof(double));
    L->N = calloc((size_t)nx * (ny + 1), sizeof(double));
    L->N2 = calloc((size_t)nx * (ny + 1), sizeof(double));
}

static void free_level(ora_level *L)
{
    free(L->h); free(L->eta); free(L->zmax); free(L->clip);
    free(L->M); free(L->M2); free(L->N); free(L->N2);
}

static int finite_all(const double *a, size_t n)
{
    for (size_t k = 0; k < n; k++)
        if (!isfinite(a[k])) return 0;
    return 1;
}

int main(void)
{
    ora_level lv[2] = {{0}};
    alloc_level(&lv[0], 40, 33);
    alloc_level(&lv[1], 36, 27);            /* 12 x 9 parent cells */
    lv[0].parent = -1;
    lv[0].dx = 810.0;
    lv[1].parent = 0;
    lv[1].off_i = 22;
    lv[1].off_j = 12;
    lv[1].dx = 270.0;
    lv[1].ox = 22 * 810.0;
    lv[1].oy = 12 * 810.0;
    uint8_t *mask = malloc((size_t)36 * 27);
    for (int j = 0; j < 27; j++)
        for (int i = 0; i < 36; i++) mask[(size_t)j * 36 + i] = !(i >= 18 && j >= 15);   /* parent cells (6.., 5..) out */
    lv[1].mask = mask;
    for (int l = 0; l < 2; l++) {
        ora_level *L = &lv[l];
        for (int j = 0; j < L->ny; j++)
            for (int i = 0; i < L->nx; i++) {
                const double x = L->ox + (i + 0.5) * L->dx;
                L->h[(size_t)j * L->nx + i] = 120.0 - x * (125.0 / 30000.0);   /* shore near x = 28.8 km */
            }
    }
    ora_domain d = {2, {0, 0, 1, 1}, lv, 1.0, 9.81, 0.025, 0.01, 0};
    ora_set_source(&d, 12000.0, 13000.0, 8000.0, 5000.0, 0.3, 2.0, 1);
    ora_step(&d, 300);
    for (int l = 0; l < 2; l++) {
        const ora_level *L = &lv[l];
        if (!finite_all(L->eta, (size_t)L->nx * L->ny) || !finite_all(L->M, (size_t)(L->nx + 1) * L->ny)
            || !finite_all(L->N, (size_t)L->nx * (L->ny + 1))) {
            fprintf(stderr, "non-finite state on level %d\n", l);
            return 1;
        }
    }
    double s = 0.0;
    for (int k = 1; k <= 20000; k++) s += ora_cbrt_rn(1.0 / (0.01 + 0.3 * k));
    s += ora_cbrt_rn(nextafter(1.0, 0.0)) + ora_cbrt_rn(8.0) + ora_cbrt_rn(nextafter(2.0, 4.0)) + ora_cbrt_rn(0x1p-1000);
    if (!isfinite(s)) return 1;
    for (int l = 0; l < 2; l++) free_level(&lv[l]);
    free(mask);
    printf("oracle ok: %lld steps\n", (long long)d.steps);
    return 0;
}
