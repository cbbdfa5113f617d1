// Dense products of the randomized eigendecomposition that the paper runs
// on top of the bbFMM matvec (Section 4, the geostatistics application):
// with l right-hand sides the range basis Q is N x l, and the algorithm
// needs Q^T Q and Q^T (K Q) (l x l, reductions over all N rows) and Q R
// (N x l times l x l).  Inputs are FP32 (what the matvec produces and
// consumes), accumulation is FP64.
//
// A^T B is split over row chunks of kChunk rows: one workgroup per (chunk,
// 16 x 16 output tile) writes its partial sum, and a second kernel adds the
// chunks' partials in chunk order, so the result does not depend on the
// launch.
#include "common.h"

namespace bbfmm {
namespace {

constexpr int kT = 16;              // output tile edge; 256 threads per tile
constexpr int kChunk = 4096;        // rows per partial product of A^T B
constexpr int kDenseMax = 1024;     // largest m or k accepted

// part[c][i][j] = sum over the rows q of chunk c of A[q][i] B[q][j]
__global__ void __launch_bounds__(256)
k_atb_part(const float *A, const float *B, int64_t n, int m, double *part) {
    __shared__ double As[kT][kT + 1], Bs[kT][kT + 1];
    const int tx = threadIdx.x & (kT - 1), ty = threadIdx.x / kT;
    const int i0 = blockIdx.z * kT, j0 = blockIdx.y * kT;
    const int64_t q0 = int64_t(blockIdx.x) * kChunk;
    const int64_t q1 = min(n, q0 + kChunk);
    double acc = 0.0;
    for (int64_t qb = q0; qb < q1; qb += kT) {
        const int64_t q = qb + ty;      // this thread stages row q, column tx of both tiles
        As[ty][tx] = (q < q1 && i0 + tx < m) ? double(A[q * m + i0 + tx]) : 0.0;
        Bs[ty][tx] = (q < q1 && j0 + tx < m) ? double(B[q * m + j0 + tx]) : 0.0;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kT; ++kk) acc = fma(As[kk][ty], Bs[kk][tx], acc);
        __syncthreads();
    }
    if (i0 + ty < m && j0 + tx < m) part[(int64_t(blockIdx.x) * m + i0 + ty) * m + j0 + tx] = acc;
}

// C[e] = sum over c = 0 .. nc-1 of part[c][e], in that order
__global__ void __launch_bounds__(256)
k_sum_parts(const double *part, int nc, int64_t len, double *C) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= len) return;
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += part[int64_t(c) * len + e];
    C[e] = s;
}

// C[q][j] = sum over i of A[q][i] R[i][j] (A n x m FP32, R m x k FP64, C n x k FP32)
__global__ void __launch_bounds__(256)
k_ab(const float *A, int64_t n, int m, const double *R, int k, float *C) {
    __shared__ double As[kT][kT + 1], Rs[kT][kT + 1];
    const int tx = threadIdx.x & (kT - 1), ty = threadIdx.x / kT;
    const int64_t q = int64_t(blockIdx.x) * kT + ty;
    const int j = blockIdx.y * kT + tx;
    double acc = 0.0;
    for (int i0 = 0; i0 < m; i0 += kT) {
        As[ty][tx] = (q < n && i0 + tx < m) ? double(A[q * m + i0 + tx]) : 0.0;
        Rs[ty][tx] = (i0 + ty < m && j < k) ? R[int64_t(i0 + ty) * k + j] : 0.0;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kT; ++kk) acc = fma(As[ty][kk], Rs[kk][tx], acc);
        __syncthreads();
    }
    if (q < n && j < k) C[q * k + j] = float(acc);
}

bool on_device(const void *ptr) {
    hipPointerAttribute_t attr{};
    return ptr != nullptr && hipPointerGetAttributes(&attr, ptr) == hipSuccess &&
           (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
}

}  // namespace
}  // namespace bbfmm

using namespace bbfmm;

extern "C" {

bbfmm_status bbfmm_dense_atb(const float *A, const float *B, int64_t n, int32_t m, double *C,
                             const bbfmm_allocator *allocator, void *stream) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(A != nullptr && B != nullptr && C != nullptr, "NULL argument");
        BB_REQUIRE(n >= 1, "n must be >= 1");
        BB_REQUIRE(m >= 1 && m <= kDenseMax, "m must be in [1, %d]", kDenseMax);
        BB_REQUIRE(allocator == nullptr || (allocator->alloc && allocator->free),
                   "allocator needs both alloc and free");
        BB_REQUIRE(on_device(A) && on_device(B) && on_device(C), "A, B and C must be device pointers");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int nc = int(ceil_div(n, kChunk));
        MemScope scope(allocator, s);
        DBuf<double> part(size_t(nc) * m * m);
        const int tiles = int(ceil_div(m, kT));
        k_atb_part<<<dim3(unsigned(nc), unsigned(tiles), unsigned(tiles)), 256, 0, s>>>(A, B, n, m, part.p);
        BB_LAUNCH_CHECK();
        const int64_t len = int64_t(m) * m;
        k_sum_parts<<<unsigned(ceil_div(len, 256)), 256, 0, s>>>(part.p, nc, len, C);
        BB_LAUNCH_CHECK();
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        return BBFMM_ERR_OUT_OF_MEMORY;
    }
}

bbfmm_status bbfmm_dense_ab(const float *A, int64_t n, int32_t m, const double *R, int32_t k,
                            float *C, void *stream) {
    bbfmm::clear_error();
    try {
        BB_REQUIRE(A != nullptr && R != nullptr && C != nullptr, "NULL argument");
        BB_REQUIRE(n >= 1, "n must be >= 1");
        BB_REQUIRE(m >= 1 && m <= kDenseMax && k >= 1 && k <= kDenseMax,
                   "m and k must be in [1, %d]", kDenseMax);
        BB_REQUIRE(on_device(A) && on_device(R) && on_device(C), "A, R and C must be device pointers");
        BB_REQUIRE(ceil_div(n, kT) <= 0x7fffffff, "n too large");
        hipStream_t s = static_cast<hipStream_t>(stream);
        k_ab<<<dim3(unsigned(ceil_div(n, kT)), unsigned(ceil_div(k, kT))), 256, 0, s>>>(A, n, m, R, k, C);
        BB_LAUNCH_CHECK();
        return BBFMM_OK;
    } catch (const Exception &e) {
        return e.status;
    }
}

}  // extern "C"
