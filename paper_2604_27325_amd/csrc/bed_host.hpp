// bed_host.hpp -- host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "../../include/bed.h"
#include "bed_internal.hpp"

namespace bed {

bed_status fail(bed_status st, const char *fmt, ...);
bed_status hip_fail(hipError_t e, const char *what);
size_t dtype_size(bed_dtype dt);
bed_status check_sizes(bed_dtype dt, int64_t batch, const int32_t *n, int nmax = 64);
bed_status check_ptr(const void *p, bed_dtype dt, const char *name, bool nullable);
bool stream_capturing(hipStream_t s);
int device_cu_count();
int size_class(int n);
TeamShape class_shape(int cls, const bed_tune &t);
bed_tune default_tune();

// Autotuner cache lookup: the stored schedule for this (arch, dtype, size mix)
// or the default one.  Never launches work.
bed_tune tuned_or_default(bed_dtype dt, int64_t batch, const int32_t *n);

bed_status plan_run_impl(const bed_plan *p, const void *A, void *lam, void *Q, int32_t *info,
                         hipStream_t s);

// Uniform batch of order 64 < n <= NMAX_BIG (binary32): reduction and tearing
// kernel, the two halves on the n <= 64 kernels, top-merge kernel.  Q may be
// NULL (eigenvalues only).
bed_status big_solve(bed_dtype dt, int64_t batch, int n, const void *A, void *lam, void *Q,
                     int32_t *info, hipStream_t s);

// Runs `launch(items, count, nmax)` with the cached device work list of a
// mixed-size batch (input order), recording its use on stream s.
bed_status with_worklist(bed_dtype dt, int64_t batch, const int32_t *n, hipStream_t s,
                         const std::function<hipError_t(const WorkItem *, int, int)> &launch);

}  // namespace bed
