// Dense kernels of the coarsest level (gfx950).
//
// The coarsest-level solve of the V-cycle is a fixed number of smoother
// sweeps from zero (paper Section 2.3: a simple iteration on the coarsest
// grid), hence a fixed linear map x = C f on a level of a few thousand cells.
// Its matrix is formed once per set of coefficients; each V-cycle then applies
// it with one matrix-vector product, a bandwidth-bound pass over n*n values
// spread over every CU, instead of a long chain of dependent sweeps on a
// single block.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mgk {
namespace {

// One wavefront per row; four independent partial sums per lane, combined in
// a fixed order, then a butterfly over the wavefront.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_matvec(const T* __restrict__ A, long long n,
                                                         const T* __restrict__ f,
                                                         T* __restrict__ x) {
    const long long row = (long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;   // wave-uniform
    const T* a = A + row * n;
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    long long j = lane;
    for (; j + 192 < n; j += 256) {
        s0 += a[j] * f[j];
        s1 += a[j + 64] * f[j + 64];
        s2 += a[j + 128] * f[j + 128];
        s3 += a[j + 192] * f[j + 192];
    }
    for (; j < n; j += 64) s0 += a[j] * f[j];
    T s = (s0 + s1) + (s2 + s3);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) x[row] = s;
}

// 32 x 32 tiles through LDS (padded against bank conflicts); 256 threads as
// 32 columns x 8 rows.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_transpose(const T* __restrict__ A,
                                                      T* __restrict__ B, long long n) {
    __shared__ T tile[32][33];
    const long long c0 = (long long)blockIdx.x * 32, r0 = (long long)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const long long i = r0 + r, j = c0 + tx;
        if (i < n && j < n) tile[r][tx] = A[i * n + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const long long i = c0 + r, j = r0 + tx;
        if (i < n && j < n) B[i * n + j] = tile[tx][r];
    }
}

}  // namespace

template <typename T>
void dense_matvec(const T* A, long long n, const T* f, T* x, hipStream_t s) {
    constexpr int rows_per_block = kBlock / 64;
    const long long nb = (n + rows_per_block - 1) / rows_per_block;
    k_dense_matvec<T><<<int(nb), kBlock, 0, s>>>(A, n, f, x);
}

template <typename T>
void transpose_square(const T* A, T* B, long long n, hipStream_t s) {
    const unsigned t = unsigned((n + 31) / 32);
    k_transpose<T><<<dim3(t, t), kBlock, 0, s>>>(A, B, n);
}

template void dense_matvec<float>(const float*, long long, const float*, float*, hipStream_t);
template void dense_matvec<double>(const double*, long long, const double*, double*,
                                   hipStream_t);
template void transpose_square<double>(const double*, double*, long long, hipStream_t);

}  // namespace mgk
