// bed_internal.hpp -- interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bed.h"

namespace bed {

// One matrix of a work list: packed offsets, size, position in the batch.
struct WorkItem {
    int64_t offA;  // element offset of A_b (and Q_b)
    int64_t offL;  // element offset of lambda_b
    int32_t n;
    int32_t idx;   // batch index (for info)
};

// One matrix of a serving step: absolute device pointers (requests own
// separate buffers).
struct PtrItem {
    const void *A;
    void *lam;
    void *Q;
    int32_t *info;
    int32_t n;
    int32_t pad;
};

// Size classes: a team of `nt` threads solves matrices with n <= nmax,
// splitting the tridiagonal matrix down to leaves of at most `leaf` elements
// (2, 4 or 8).  Default cutoff per class (measured on the batch-512
// workloads): 8 for the n > 32 class, whose one fewer merge depth outweighs
// the longer Jacobi sweeps, 4 below.
__host__ __device__ constexpr int leaf_default(int nmax) { return nmax >= 64 ? 8 : 4; }
struct TeamShape {
    int nmax;
    int nt;
    int leaf = 4;
};
inline bool leaf_supported(int leaf) { return leaf == 2 || leaf == 4 || leaf == 8; }

// Largest order of the one-shot solve (64 < n <= NMAX_BIG: binary32, uniform
// batches, one tearing step above the n <= 64 kernels).
constexpr int NMAX_BIG = 128;

bool team_supported(bed_dtype dt, TeamShape ts);

// One workgroup per matrix of a uniform batch.
hipError_t launch_uniform(bed_dtype dt, TeamShape ts, const void *A, int n, int64_t batch,
                          void *lam, void *Q, int32_t *info, hipStream_t s);

// Uniform batch of binary32 tridiagonal matrices (diagonal then off-diagonal,
// 2n values apart); team shapes (32, 128), (32, 256) and (64, 512).  With Q == nullptr
// (eigenvalues only) ends, if not null, receives each matrix's first and last
// eigenvector rows (2n values apart).
hipError_t launch_tri(TeamShape ts, const float *tri, int n, int64_t batch, float *lam, float *Q,
                      int32_t *info, float *ends, hipStream_t s);

// Work-list launch.  counter == nullptr: workgroup i handles items i, i+grid,
// ... (static).  counter != nullptr: persistent workgroups pull items from
// counter[0]; counter[1] counts finished workgroups and the last one resets
// both to zero, so the launch can be replayed (e.g. from a HIP graph).
hipError_t launch_list(bed_dtype dt, TeamShape ts, const void *A, void *lam, void *Q,
                       int32_t *info, const WorkItem *items, int count, int *counter, int grid,
                       hipStream_t s);

// One workgroup per pointer item (serving steps).
hipError_t launch_ptrlist(bed_dtype dt, TeamShape ts, const PtrItem *items, int count,
                          hipStream_t s);

// Resident workgroups per CU for a team shape (occupancy query).
int blocks_per_cu(bed_dtype dt, TeamShape ts);

// Backward kernel over a work list (one workgroup per matrix).
hipError_t launch_backward(bed_dtype dt, int nmax, const void *lam, const void *Q,
                           const void *dlam, const void *dQ, void *dA, const WorkItem *items,
                           int count, double eps, hipStream_t s);
hipError_t launch_backward_uniform(bed_dtype dt, int nmax, const void *lam, const void *Q,
                                   const void *dlam, const void *dQ, void *dA, int n,
                                   int64_t batch, double eps, hipStream_t s);

}  // namespace bed
