/*
 * rpba_testing.h -- test-only entry points of librpba.  Not part of the
 * method's interface (include/rpba.h); the parity tests use them to check
 * building blocks of the kernels in isolation.
 */
#ifndef RPBA_TESTING_H
#define RPBA_TESTING_H

#include "rpba.h"

#ifdef __cplusplus
extern "C" {
#endif

/* FP64 matrix-core tile product of the dense Cholesky (Sec. 2: the reduced
 * camera system is factorised): C = A B^T for 64 x 64 row-major DEVICE
 * tiles, one workgroup on `stream` (a hipStream_t, NULL = default).  Returns
 * RPBA_ERR_HIP if the launch fails. */
rpba_status rpba_selftest_gemm(const double *A, const double *B, double *C, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RPBA_TESTING_H */
