// gaussian.hip -- the random operators of the randomization step (Sec. 2):
// the Gaussian sketch operator G, the subsampled randomized Fourier operator
// S F D of eqs. (4)-(7), and the power-iteration start vector; plus a fill
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

// S F D written out: row i keeps frequency s_i of the unnormalised DFT of
// D A, so G(i, p) = exp(2 pi i (phi_p - (s_i p mod m) / m)), with phi_p the
// first uniform of Philox counter (p, 0, 0, 5) and s_i = floor(u m) for the
// first uniform u of counter (i, 0, 0, 6) (i.i.d., with replacement).

__global__ __launch_bounds__(256) void srft_kernel(int64_t rows, int64_t m, uint64_t seed,
                                                   double2 *out, int64_t ld) {
  const int64_t total = rows * m;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / m;
    const int64_t p = e - i * m;
    int64_t si = static_cast<int64_t>(floor(rid_u1(seed, 6u, static_cast<uint64_t>(i)) *
                                            static_cast<double>(m)));
    if (si >= m) si = m - 1;
    const int64_t r = static_cast<int64_t>((static_cast<uint64_t>(si) * static_cast<uint64_t>(p)) %
                                           static_cast<uint64_t>(m));
    const double ang = 6.283185307179586476925286766559 *
                       (rid_u1(seed, 5u, static_cast<uint64_t>(p)) -
                        static_cast<double>(r) / static_cast<double>(m));
    out[i * ld + p] = make_double2(cos(ang), sin(ang));
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

hipError_t launch_srft(hipStream_t st, int64_t rows, int64_t m, uint64_t seed, double2 *out,
                       int64_t ld) {
  const int64_t total = rows * m;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(srft_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, rows, m,
                     seed, out, ld);
  return hipGetLastError();
}

hipError_t launch_operator(hipStream_t st, int kind, int64_t rows, int64_t cols, uint64_t seed,
                           double2 *out, int64_t ld) {
  if (kind == RID_SKETCH_SRFT) return launch_srft(st, rows, cols, seed, out, ld);
  return launch_gaussian(st, rows, cols, seed, 0, out, ld);
}
