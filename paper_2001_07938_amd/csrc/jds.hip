// CSR -> JDS conversion on the device.
//
// Jagged Diagonal Storage (the paper's section "Sparse Matrix Variations in
// LiLAC-What", JDS paragraph and the JDS figure): the rows are put in order
// of decreasing non-zero count, ties kept in their original order; perm[i]
// is the new position of original row i, nzcnt[p] the count of the row at
// position p; diagonal j holds the j-th entry of every row that has one, in
// position order, starting at jd_ptr[j], so entry j of the row at position
// p sits at jd_ptr[j] + p.
//
// Steps, each one launch on the caller's stream:
//   1. the longest row (an integer maximum, read back to size the rest);
//   2. keys max_len - len_i with values i, sorted by a stable device radix
//      sort (rocPRIM), which gives the rows in order of decreasing length
//      and ascending index among equal lengths;
//   3. perm and nzcnt from the sorted order;
//   4. per diagonal j the number of rows longer than j (a binary search in
//      the non-increasing nzcnt), then an exclusive scan into jd_ptr;
//   5. every CSR entry scattered to jd_ptr[j] + perm[row]: reads stream
//      through the CSR arrays, each entry is written once.
// Everything is integer or a copy of a value, so the result is exact.
#include <rocprim/device/device_radix_sort.hpp>

#include "lilac_internal.h"

namespace lilac {
namespace {

constexpr int kT = 256;

inline int32_t blocks_for(int64_t n)
{
    const int64_t b = (n + kT - 1) / kT;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 20));
}

__global__ __launch_bounds__(kT) void k_row_len_max(int32_t rows,
                                                    const int32_t *__restrict__ rp,
                                                    int32_t *__restrict__ out)
{
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * kT)
        m = max(m, rp[i + 1] - rp[i]);
    // wavefront maximum, then one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1)
        m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0)
        atomicMax(out, m);
}

__global__ __launch_bounds__(kT) void k_jds_keys(int32_t rows, const int32_t *__restrict__ rp,
                                                 int32_t max_len, uint32_t *__restrict__ key,
                                                 int32_t *__restrict__ idx)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * kT) {
        key[i] = (uint32_t)(max_len - (rp[i + 1] - rp[i]));
        idx[i] = (int32_t)i;
    }
}

__global__ __launch_bounds__(kT) void k_jds_perm(int32_t rows, int32_t max_len,
                                                 const uint32_t *__restrict__ key,
                                                 const int32_t *__restrict__ order,
                                                 int32_t *__restrict__ perm,
                                                 int32_t *__restrict__ nzcnt)
{
    for (int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x; p < rows;
         p += (int64_t)gridDim.x * kT) {
        perm[order[p]] = (int32_t)p;
        nzcnt[p] = max_len - (int32_t)key[p];
    }
}

// cnt[j] = #{p : nzcnt[p] > j} for j < max_len (nzcnt is non-increasing, so
// that is the first position whose count is <= j); cnt[max_len] = 0 so that
// the exclusive scan of cnt[0..max_len] ends with the number of entries.
__global__ __launch_bounds__(kT) void k_jds_diag_count(int32_t rows, int32_t max_len,
                                                       const int32_t *__restrict__ nzcnt,
                                                       int32_t *__restrict__ cnt)
{
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j <= max_len;
         j += (int64_t)gridDim.x * kT) {
        if (j == max_len) {
            cnt[j] = 0;
            continue;
        }
        int32_t lo = 0, hi = rows;   // first p in [lo, hi) with nzcnt[p] <= j
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (nzcnt[mid] > j)
                lo = mid + 1;
            else
                hi = mid;
        }
        cnt[j] = lo;
    }
}

template <typename V>
__global__ __launch_bounds__(kT) void k_jds_scatter(
    int32_t rows, int64_t nnz, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const V *__restrict__ vals,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ jd_ptr,
    int32_t *__restrict__ jd_col, V *__restrict__ jd_val)
{
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kT) {
        // the row holding entry e: the last i with rp[i] <= e
        int32_t lo = 0, hi = rows - 1;
        while (lo < hi) {
            const int32_t mid = hi - (hi - lo) / 2;
            if (rp[mid] <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int32_t j = (int32_t)(e - rp[lo]);
        const int64_t k = (int64_t)jd_ptr[j] + perm[lo];
        jd_col[k] = col[e];
        jd_val[k] = vals[e];
    }
}

}  // namespace

int32_t jds_max_len(const CsrHandle &h, int32_t *d_tmp, hipStream_t s)
{
    if (h.rows == 0)
        return 0;
    launch_fill_i32(d_tmp, 1, 0, s);
    hipLaunchKernelGGL(k_row_len_max, dim3(blocks_for(h.rows)), dim3(kT), 0, s, h.rows,
                       h.d_row_ptr, d_tmp);
    HIPC(hipGetLastError());
    int32_t m = 0;
    HIPC(hipMemcpyAsync(&m, d_tmp, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return m;
}

void jds_convert(const CsrHandle &h, int32_t max_len, int32_t *perm, int32_t *nzcnt,
                 int32_t *jd_ptr, int32_t *jd_col, void *jd_val, hipStream_t s)
{
    const int32_t rows = h.rows;
    if (rows == 0) {
        launch_fill_i32(jd_ptr, 1, 0, s);
        return;
    }
    // sort buffers: keys and row indices in and out, plus rocPRIM's scratch
    uint32_t *key_in = (uint32_t *)dev_alloc((size_t)rows * 4);
    uint32_t *key_out = nullptr;
    int32_t *idx_in = nullptr, *idx_out = nullptr;
    void *tmp = nullptr;
    try {
        key_out = (uint32_t *)dev_alloc((size_t)rows * 4);
        idx_in = (int32_t *)dev_alloc((size_t)rows * 4);
        idx_out = (int32_t *)dev_alloc((size_t)rows * 4);
        hipLaunchKernelGGL(k_jds_keys, dim3(blocks_for(rows)), dim3(kT), 0, s, rows,
                           h.d_row_ptr, max_len, key_in, idx_in);
        HIPC(hipGetLastError());
        int end_bit = 0;
        while (end_bit < 32 && ((uint32_t)max_len >> end_bit) != 0)
            ++end_bit;
        if (end_bit > 0) {
            size_t bytes = 0;
            HIPC(rocprim::radix_sort_pairs(nullptr, bytes, key_in, key_out, idx_in, idx_out,
                                           (size_t)rows, 0, end_bit, s));
            tmp = dev_alloc(std::max<size_t>(bytes, 4));
            HIPC(rocprim::radix_sort_pairs(tmp, bytes, key_in, key_out, idx_in, idx_out,
                                           (size_t)rows, 0, end_bit, s));
        } else {
            // every row is empty: the order is the identity
            HIPC(hipMemcpyAsync(key_out, key_in, (size_t)rows * 4, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(idx_out, idx_in, (size_t)rows * 4, hipMemcpyDeviceToDevice, s));
        }
        hipLaunchKernelGGL(k_jds_perm, dim3(blocks_for(rows)), dim3(kT), 0, s, rows, max_len,
                           (const uint32_t *)key_out, (const int32_t *)idx_out, perm, nzcnt);
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_jds_diag_count, dim3(blocks_for((int64_t)max_len + 1)), dim3(kT),
                           0, s, rows, max_len, (const int32_t *)nzcnt, jd_ptr);
        HIPC(hipGetLastError());
        launch_scan_excl(jd_ptr, (int64_t)max_len + 1, nullptr, s);
        if (h.nnz > 0) {
            if (h.dt == LILAC_F32)
                hipLaunchKernelGGL(k_jds_scatter<float>, dim3(blocks_for(h.nnz)), dim3(kT), 0,
                                   s, rows, h.nnz, h.d_row_ptr, h.d_col,
                                   (const float *)h.d_vals, (const int32_t *)perm,
                                   (const int32_t *)jd_ptr, jd_col, (float *)jd_val);
            else
                hipLaunchKernelGGL(k_jds_scatter<double>, dim3(blocks_for(h.nnz)), dim3(kT), 0,
                                   s, rows, h.nnz, h.d_row_ptr, h.d_col,
                                   (const double *)h.d_vals, (const int32_t *)perm,
                                   (const int32_t *)jd_ptr, jd_col, (double *)jd_val);
            HIPC(hipGetLastError());
        }
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dev_free(key_in);
        dev_free(key_out);
        dev_free(idx_in);
        dev_free(idx_out);
        dev_free(tmp);
        throw;
    }
    dev_free(key_in);
    dev_free(key_out);
    dev_free(idx_in);
    dev_free(idx_out);
    dev_free(tmp);
}

}  // namespace lilac
