// gaussian.hip -- the Gaussian draws of the randomization step (Sec. 2):
// the sketch operator G and the power-iteration start vector; plus a fill
// kernel for the empty-sum case of the sketch.
#include "rid_internal.hpp"

namespace {

// One thread per entry, grid-stride over rows * cols, row-major output.
__global__ __launch_bounds__(256) void gaussian_kernel(int64_t rows, int64_t cols,
                                                       uint64_t seed, uint32_t stream_id,
                                                       double2 *out, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / cols;
    const int64_t j = e - i * cols;
    out[i * ld + j] = rid_gauss(seed, stream_id, static_cast<uint32_t>(i),
                                static_cast<uint64_t>(j));
  }
}

// Zero an l x n complex128 block with leading dimension ld.
__global__ __launch_bounds__(256) void zero_kernel(int64_t rows, int64_t cols, double2 *out,
                                                   int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = e / rows;
    out[j * ld + (e - j * rows)] = make_double2(0.0, 0.0);
  }
}

}  // namespace

hipError_t launch_zero(hipStream_t st, int64_t rows, int64_t cols, double2 *out, int64_t ld) {
  const int64_t total = rows * cols;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, rows,
                     cols, out, ld);
  return hipGetLastError();
}

hipError_t launch_gaussian(hipStream_t st, int64_t rows, int64_t cols, uint64_t seed,
                           uint32_t stream_id, double2 *out, int64_t ld) {
  const int64_t total = rows * cols;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gaussian_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     rows, cols, seed, stream_id, out, ld);
  return hipGetLastError();
}
