/* A plain C99 user of the C ABI: only host entry points that need no GPU
 * (version, argument errors, the tridiagonal eigenvalue utility).  Prints
 * "ok" and returns 0 on success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "csl.h"

int main(void) {
    if (csl_version() < 200) return 1;
    /* tridiag(1, 2, 1) of order 3: eigenvalues 2 - sqrt 2, 2, 2 + sqrt 2 */
    const double d[3] = {2.0, 2.0, 2.0}, e[2] = {1.0, 1.0};
    double th[3];
    if (csl_tridiagonal_eigenvalues(d, e, 3, th) != CSL_OK) return 2;
    const double want[3] = {2.0 - sqrt(2.0), 2.0, 2.0 + sqrt(2.0)};
    for (int i = 0; i < 3; ++i)
        if (fabs(th[i] - want[i]) > 1e-14) return 3;
    /* validation fails before any device work */
    csl_problem p = NULL;
    if (create_problem(NULL, NULL, 1.0, 1.0, NULL, 0, &p) != CSL_ERR_ARG || p != NULL) return 4;
    if (strlen(csl_last_error()) == 0) return 5;
    csl_grid g = {2, {7, 1500, 0}, {1.0, 1.0, 0.0}};
    if (create_problem(&g, (const double *)0x1000, 1.0, 1.0, NULL, 0, &p) != CSL_ERR_ARG) return 6;
    printf("ok\n");
    return 0;
}
