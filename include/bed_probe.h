/*
 * bed_probe.h -- instrumented copy of the uniform-batch solver, for
 * measurement only (library libbed_probe.so, never used by the product
 * entry points).  The kernel code is the solver's own, compiled with
 * timestamps at its phase boundaries and inside one Householder step.
 */
#ifndef BED_PROBE_H
#define BED_PROBE_H

#include <stdint.h>

#define BED_PROBE_PHASES 64   /* phase marks per team                      */
#define BED_PROBE_SUBSTEPS 16 /* sub-step marks of the chosen Householder step */

#ifdef __cplusplus
extern "C" {
#endif

/* Solves `batch` matrices of order n (uniform, packed as in bed.h, FP32 when
 * dtype == 0 else FP64) with `threads` threads per matrix (the supported team
 * shapes of bed.h) and records:
 *   marks[b*64 + id]  100 MHz real-time clock of team b at phase boundary id
 *                     (0 where the phase does not occur): 0 start, 1 loaded,
 *                     2 Householder done, 3 leaves done, 10+8d+j merge phases
 *                     of depth d (j = 0 setup, 1 roots, 2 Loewner, 3 vectors,
 *                     4 rotations, 5 back-multiplication), 4 back-transform
 *                     done, 5 stored;
 *   steps[b*16 + id]  shader-clock cycles at sub-step id of the middle
 *                     Householder step (k = 32 for n > 32, 16 for 16 < n <= 32,
 *                     8 below) in wave 0: 0 start, 1 dot product, 2 partial
 *                     exchange and barrier, 3 reduction p^T v, 4 w broadcast,
 *                     5 reduction of the pivot column norm, 6 reflector,
 *                     7 v broadcast writes, 8 rank-2 update, 9 a
 *                     second stamp right after 8 (the cost of one marker,
 *                     which waits for outstanding LDS and scalar operations).
 *   defl[b*2 + t]     (may be NULL) deflations of team b summed over its merge
 *                     depths: t = 0 type 1 (rho |z_i| <= tol), t = 1 type 2
 *                     (Givens rotation of a close pair of poles).
 * marks, steps and defl are device arrays of batch*64, batch*16 and batch*2
 * int64 values; they are cleared first.  Synchronizes `stream` before the launch (the
 * buffer addresses are copied from host locals).  Returns 0 on success, 1 for
 * an invalid argument, 3 for a HIP failure. */
int32_t bed_probe_phases(int32_t dtype, int32_t threads, int32_t n, int64_t batch,
                         const void *A, void *lambda, void *Q, long long *marks,
                         long long *steps, long long *defl, void *stream);

#ifdef __cplusplus
}
#endif
#endif
