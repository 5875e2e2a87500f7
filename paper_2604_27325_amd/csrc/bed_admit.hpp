// bed_admit.hpp -- admission accounting of the request server: a request of
// `count` matrices of order n is admitted while the matrices in flight and the
// bytes of admitted request buffers stay within their limits (0 = no limit).
// Host code only (no HIP), so the policy is testable without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace bed {

// Bytes of one request's buffers: A and Q (n x n each) and lambda (n) per
// matrix, at `elem` bytes per element.
inline int64_t request_bytes(int32_t count, int32_t n, size_t elem)
{
    return (int64_t)count * (2 * (int64_t)n * n + n) * (int64_t)elem;
}

enum AdmitResult { ADMIT_OK = 0, ADMIT_INFLIGHT = 1, ADMIT_MEMORY = 2 };

struct Admission {
    int64_t max_mats = 0;   // matrices in flight (0: unlimited)
    int64_t max_bytes = 0;  // bytes of admitted request buffers (0: unlimited)
    int64_t mats = 0, bytes = 0;

    // Admits (and accounts) the request or reports which limit refuses it.
    AdmitResult admit(int64_t count, int64_t nbytes)
    {
        if (max_mats > 0 && mats + count > max_mats) return ADMIT_INFLIGHT;
        if (max_bytes > 0 && bytes + nbytes > max_bytes) return ADMIT_MEMORY;
        mats += count;
        bytes += nbytes;
        return ADMIT_OK;
    }
    // A completed request returns its share.
    void release(int64_t count, int64_t nbytes)
    {
        mats -= count;
        bytes -= nbytes;
    }
    bool idle() const { return mats == 0; }
};

}  // namespace bed
