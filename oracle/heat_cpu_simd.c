/*
 * heat_cpu_simd.c -- the segment sweep of the paper's threaded CPU method,
 * vectorised.  TEST AND MEASUREMENT INFRASTRUCTURE, like heat_oracle.c, which
 * calls it: only the test suite and the benchmark's CPU legs load it.
 *
 * Beside its scalar codes the paper wrote a SIMD-vectorised build of its Rust
 * solver, faster with few threads and less so as threads are added, and
 * measured the scalar ones (Section 3, Rust; Section 4 on SIMD in each
 * language).  This is the SIMD counterpart of the scalar sweep in
 * heat_oracle.c.  It
 * evaluates each cell with exactly the same binary64 operations in the same
 * order (Section 2, Eq. (heat:discrete), with r = alpha*dt/h^2):
 *         new = c + r * ((l - 2.0 * c) + q)
 * and only lets the compiler run several cells per instruction.  The file is
 * built with -O3 -ffp-contract=off -fno-fast-math, so no operation is fused
 * or reassociated and the result is bit-identical to the scalar sweep.  The
 * function is cloned for AVX-512F, AVX2 and baseline x86-64 and the loader
 * picks the clone the running CPU supports.
 */
#include <stdint.h>

void heat_cpu_sweep_simd(const double *restrict a, double *restrict b, int64_t len, double r);

__attribute__((target_clones("avx512f", "avx2", "default")))
void heat_cpu_sweep_simd(const double *restrict a, double *restrict b, int64_t len, double r)
{
    /* a[0] and a[len + 1] are the ghost cells; b[1..len] is written */
    for (int64_t j = 1; j <= len; ++j)
        b[j] = a[j] + r * ((a[j - 1] - 2.0 * a[j]) + a[j + 1]);
}
