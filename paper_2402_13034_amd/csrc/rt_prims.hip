// Sorting, de-duplication and scans of integer keys on the device (rocPRIM).
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "rt_host.hpp"

namespace rt {

// device (or managed) memory, as opposed to host memory, pinned or not
bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// keys_in sorted into keys_out (n >= 1; keys_in is left in an unspecified order)
void sort_u64_into(Ctx& c, uint64_t* keys_in, uint64_t* keys_out, int64_t n, int end_bit, hipStream_t st)
{
    if (n == 1) {
        HIP_CHECK(hipMemcpyAsync(keys_out, keys_in, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        return;
    }
    if (n <= 0) return;
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_keys(nullptr, bytes, keys_in, keys_out, (size_t)n, 0, end_bit, st));
    Scratch tmp(c, bytes, st);
    HIP_CHECK(rocprim::radix_sort_keys(tmp.p, bytes, keys_in, keys_out, (size_t)n, 0, end_bit, st));
}

void sort_u64(Ctx& c, uint64_t* keys, int64_t n, int end_bit, hipStream_t st)
{
    if (n <= 1) return;
    Scratch tmp_keys(c, sizeof(uint64_t) * (size_t)n, st);
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_keys(nullptr, bytes, keys, tmp_keys.as<uint64_t>(), (size_t)n, 0,
                                       end_bit, st));
    Scratch tmp(c, bytes, st);
    HIP_CHECK(rocprim::radix_sort_keys(tmp.p, bytes, keys, tmp_keys.as<uint64_t>(), (size_t)n, 0,
                                       end_bit, st));
    HIP_CHECK(hipMemcpyAsync(keys, tmp_keys.p, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
}

void unique_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t n, int64_t* d_count, hipStream_t st)
{
    size_t bytes = 0;
    HIP_CHECK(rocprim::unique(nullptr, bytes, in, out, d_count, (size_t)n, rocprim::equal_to<uint64_t>(), st));
    Scratch tmp(c, bytes, st);
    HIP_CHECK(rocprim::unique(tmp.p, bytes, in, out, d_count, (size_t)n, rocprim::equal_to<uint64_t>(), st));
}

__global__ void k_scan_total(const uint8_t* flags, const int64_t* off, int64_t n, int64_t* total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) total[0] = n > 0 ? off[n - 1] + (int64_t)flags[n - 1] : 0;
}

void scan_flags(Ctx& c, const uint8_t* flags, int64_t* offsets, int64_t n, int64_t* d_total, hipStream_t st)
{
    if (n == 0) {
        HIP_CHECK(hipMemsetAsync(d_total, 0, sizeof(int64_t), st));
        return;
    }
    auto in = rocprim::make_transform_iterator(flags, [] __device__(uint8_t f) { return (int64_t)f; });
    size_t bytes = 0;
    HIP_CHECK(rocprim::exclusive_scan(nullptr, bytes, in, offsets, (int64_t)0, (size_t)n,
                                      rocprim::plus<int64_t>(), st));
    Scratch tmp(c, bytes, st);
    HIP_CHECK(rocprim::exclusive_scan(tmp.p, bytes, in, offsets, (int64_t)0, (size_t)n,
                                      rocprim::plus<int64_t>(), st));
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, st, flags, offsets, n, d_total);
    HIP_CHECK(hipGetLastError());
}

void scan_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n, hipStream_t st)
{
    if (n == 0) return;
    size_t bytes = 0;
    HIP_CHECK(rocprim::exclusive_scan(nullptr, bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), st));
    Scratch tmp(c, bytes, st);
    HIP_CHECK(rocprim::exclusive_scan(tmp.p, bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), st));
}

}  // namespace rt
