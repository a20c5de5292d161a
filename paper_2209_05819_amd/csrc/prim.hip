// Device-wide sort and scan primitives (rocPRIM) used while building the tree
// and the lists.  Temporary storage is allocated per call: these run during
// the build only, never inside a matvec.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "hodlr_impl.hpp"

namespace hodlr {

namespace {
struct TmpBuf {
    void* p = nullptr;
    ~TmpBuf() {
        if (p) (void)hipFree(p);
    }
    void* get(size_t bytes) {
        HIP_CHECK(hipMalloc(&p, bytes ? bytes : 16));
        return p;
    }
};
}  // namespace

void sort_pairs_u64(const uint64_t* kin, uint64_t* kout, const int32_t* vin, int32_t* vout,
                    int64_t n, int end_bit, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0u,
                                        (unsigned)end_bit, s));
    TmpBuf t;
    void* tmp = t.get(bytes);
    HIP_CHECK(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)n, 0u,
                                        (unsigned)end_bit, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::exclusive_scan(nullptr, bytes, in, out, (int32_t)0, (size_t)n,
                                      rocprim::plus<int32_t>(), s));
    TmpBuf t;
    void* tmp = t.get(bytes);
    HIP_CHECK(rocprim::exclusive_scan(tmp, bytes, in, out, (int32_t)0, (size_t)n,
                                      rocprim::plus<int32_t>(), s));
    HIP_CHECK(hipStreamSynchronize(s));
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::exclusive_scan(nullptr, bytes, in, out, (int64_t)0, (size_t)n,
                                      rocprim::plus<int64_t>(), s));
    TmpBuf t;
    void* tmp = t.get(bytes);
    HIP_CHECK(rocprim::exclusive_scan(tmp, bytes, in, out, (int64_t)0, (size_t)n,
                                      rocprim::plus<int64_t>(), s));
    HIP_CHECK(hipStreamSynchronize(s));
}

void segmented_sort_i32(const int32_t* in, int32_t* out, int64_t nnz, int64_t nseg,
                        const int64_t* offsets, hipStream_t s) {
    size_t bytes = 0;
    HIP_CHECK(rocprim::segmented_radix_sort_keys(nullptr, bytes, in, out, (unsigned)nnz,
                                                 (unsigned)nseg, offsets, offsets + 1, 0u, 32u,
                                                 s));
    TmpBuf t;
    void* tmp = t.get(bytes);
    HIP_CHECK(rocprim::segmented_radix_sort_keys(tmp, bytes, in, out, (unsigned)nnz,
                                                 (unsigned)nseg, offsets, offsets + 1, 0u, 32u,
                                                 s));
    HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace hodlr
