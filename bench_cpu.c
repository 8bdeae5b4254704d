/* Multi-core host CSR product for the benchmark's CPU baseline.
 *
 * Not part of the oracle and not part of the library: the benchmark times it
 * beside the oracle's single-threaded product to report what all host cores
 * reach on the same matrix.  Rows are split into static blocks over the
 * OpenMP threads; each row is summed left to right in storage order, as the
 * oracle does, so the result is identical for every thread count.  Indices
 * are int32, as the byte count of the benchmark assumes.                     */
#include <omp.h>
#include <stdint.h>

int cpu_threads(void) { return omp_get_max_threads(); }

int cpu_csr_spmv(int32_t m, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            s = s + vals[p] * x[colidx[p]];
        y[i] = s;
    }
    return 0;
}
