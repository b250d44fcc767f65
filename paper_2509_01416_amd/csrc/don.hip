// don.hip -- elementwise and reduction kernels of the deep operator network
// (arXiv 2509.01416 section 4.1, Eq. 11): the ReLU mask of the backward
// pass, fixed-order column sums for the bias gradients, and the trunk
// network's input (cell-centre coordinates).  The dense layers run on the
// batched matrix-core GEMM of fno.hip.
#include "fno_kernels.h"

namespace mdp {

__global__ void relu_back_kernel(const float* __restrict__ z, const float* __restrict__ g,
                                 float* __restrict__ out, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        out[e] = z[e] > 0.f ? g[e] : 0.f;
}

// Stage 1: grid (ceil(C / 64), chunks); thread (column c, chunk k) sums rows
// [k * kColChunk, (k + 1) * kColChunk) of column c in row order.
__global__ void col_sum_part_kernel(const float* __restrict__ x, float* __restrict__ part,
                                    int R, int C) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (c >= C) return;
    const int r1 = min(R, (k + 1) * kColChunk);
    float s = 0.f;
    for (int r = k * kColChunk; r < r1; ++r) s += x[(size_t)r * C + c];
    part[(size_t)k * C + c] = s;
}

// Stage 2: chunk sums of a column in chunk order.
__global__ void col_sum_fin_kernel(const float* __restrict__ part, float* __restrict__ out,
                                   int nchunk, int C) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int k = 0; k < nchunk; ++k) s += part[(size_t)k * C + c];
    out[c] = s;
}

// (x/lx, y/ly) of the n x n cell centres, cell-major with x fastest.
__global__ void grid_coords_kernel(float* __restrict__ xy, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n * n) return;
    const int iy = p / n, ix = p - iy * n;
    xy[2 * p] = (ix + 0.5f) / n;
    xy[2 * p + 1] = (iy + 0.5f) / n;
}

void launch_relu_back(const float* z, const float* g, float* out, long long n, hipStream_t s) {
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(relu_back_kernel, dim3((unsigned)blocks), dim3(256), 0, s, z, g, out, n);
}

void launch_col_sum(const float* x, float* out, int R, int C, float* scratch, hipStream_t s) {
    const int nchunk = (R + kColChunk - 1) / kColChunk;
    hipLaunchKernelGGL(col_sum_part_kernel, dim3((C + 63) / 64, nchunk), dim3(64), 0, s, x,
                       scratch, R, C);
    hipLaunchKernelGGL(col_sum_fin_kernel, dim3((C + 63) / 64), dim3(64), 0, s, scratch, out,
                       nchunk, C);
}

void launch_grid_coords(float* xy, int n, hipStream_t s) {
    hipLaunchKernelGGL(grid_coords_kernel, dim3((n * n + 255) / 256), dim3(256), 0, s, xy, n);
}

}  // namespace mdp
