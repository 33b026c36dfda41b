// csr.hip — membership CSR from the appended keys (ordinal << bn | original index).
//
// Sorting the keys orders rows by landmark ordinal and columns by ascending
// original index in one pass, so the result does not depend on the order in
// which the range passes appended members.
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "dev_common.h"
#include "kernels.h"

namespace bm {

hipError_t sort_keys(void *tmp, size_t *tmp_bytes, const uint64_t *in, uint64_t *out, size_t count,
                     int end_bit, hipStream_t s)
{
    size_t bytes = *tmp_bytes;
    hipError_t e = rocprim::radix_sort_keys(tmp, bytes, in, out, count, 0u, (unsigned)end_bit, s);
    *tmp_bytes = bytes;
    return e;
}

// row_ptr[i] = first position whose key is >= i << bn (i = 0..L); member_idx = low bits.
__global__ void k_row_ptr(const uint64_t *keys, int64_t M, int64_t L, int32_t bn, int64_t *row_ptr)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > L) return;
    const uint64_t target = (uint64_t)i << bn;
    int64_t lo = 0, hi = M;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    row_ptr[i] = lo;
}

__global__ void k_member_idx(const uint64_t *keys, int64_t M, int32_t bn, int32_t *member_idx)
{
    const uint64_t mask = (bn >= 64) ? ~0ull : ((1ull << bn) - 1);
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x)
        member_idx[m] = (int32_t)(keys[m] & mask);
}

hipError_t launch_csr_from_sorted(const uint64_t *keys, int64_t M, int64_t L, int32_t bn, int64_t *row_ptr,
                                  int32_t *member_idx, hipStream_t s)
{
    k_row_ptr<<<(int)((L + 1 + 255) / 256), 256, 0, s>>>(keys, M, L, bn, row_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || M == 0) return e;
    int64_t blocks = (M + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    k_member_idx<<<(int)blocks, 256, 0, s>>>(keys, M, bn, member_idx);
    return hipGetLastError();
}

} // namespace bm
